"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds inputs: grids, densities, frequency bins, dust
tables, sources and run parameters, as plain numpy arrays in cgs units.  It
contains none of the transport, estimator or temperature arithmetic, and it
is the only module that both the oracle tests and the HIP path use.

Workloads (the paper's own data -- dust tables, benchmark results, the AMR
snapshot -- are not available, so these stand in for them):

* ``config0``: 32^3 uniform dust sphere (r < 0.9 AU, tau_ext(1 um) = 1)
  around a 5800 K, 1 L_sun star at the origin; kappa ~ nu^1 (100 cm^2/g at
  1 um), albedo 0.5, HG g = 0.6; 100 log bins over 0.1-1000 um.
* ``config1``: 128^3 flared disk (+-120 AU), rho0 (R/AU)^-1 exp(-z^2/2h^2),
  h = 0.05 R (R/AU)^0.125, 1 < R < 100 AU, radial mid-plane tau(1 um) = 1e3,
  around a 4000 K, 2 R_sun star (the shape of the Sec. 4 disk benchmarks);
  kappa ~ nu^1.5, albedo 0.5 exp(-lambda/10 um); 200 bins; images at the
  bins holding 1, 10 and 100 um.
* ``config2``: 256^3 log-normal clump from a Gaussian random field with
  P(k) ~ k^-11/3, sigma_ln rho = 1.5, mean column tau(1 um) = 50, in a
  0.65 pc box with 50 point sources (dN/dL ~ L^-1.5 on 0.1-1e3 L_sun,
  T_eff log-uniform on 3000-20000 K) -- the shape of the Sec. 5 region.
* ``config3_model(m)``: member m of the 512-model batched family.
* ``slab``: pure absorber slab for the exp(-tau) transmission pin.
"""
from __future__ import annotations

import math

import numpy as np

# physical constants used to lay out inputs (cgs; CODATA 2018, IAU 2015)
AU = 1.495978707e13
PC = 3.0857e18
L_SUN = 3.828e33
R_SUN = 6.957e10
C_LIGHT = 2.99792458e10
SIGMA_SB = 5.670374419e-5
MICRON = 1e-4


def nu_edges_log(n_bins: int, lam_min_um: float = 0.1, lam_max_um: float = 1000.0) -> np.ndarray:
    """n_bins+1 frequency edges, log-spaced in wavelength, increasing in nu."""
    lam = np.logspace(math.log10(lam_min_um), math.log10(lam_max_um), n_bins + 1) * MICRON
    return np.ascontiguousarray((C_LIGHT / lam)[::-1])


def bin_centres(nu_edges: np.ndarray) -> np.ndarray:
    """geometric-mean frequency of each bin (dust properties are taken there)"""
    return np.sqrt(nu_edges[:-1] * nu_edges[1:])


def bin_of_wavelength(nu_edges: np.ndarray, lam_um: float) -> int:
    nu = C_LIGHT / (lam_um * MICRON)
    k = int(np.searchsorted(nu_edges, nu, side="right") - 1)
    return min(max(k, 0), len(nu_edges) - 2)


def powerlaw_dust(nu_edges, beta, albedo=0.5, g=0.6, kappa_1um=100.0, albedo_fn=None):
    """kappa = kappa_1um (nu/nu_1um)^beta; chi = kappa/(1-albedo)."""
    nuc = bin_centres(nu_edges)
    nu1 = C_LIGHT / MICRON
    kappa = kappa_1um * (nuc / nu1) ** beta
    if albedo_fn is not None:
        alb = albedo_fn(C_LIGHT / nuc / MICRON)
    else:
        alb = np.full_like(nuc, albedo)
    chi = kappa / (1.0 - alb)
    return {"chi": chi, "albedo": np.asarray(alb, dtype=np.float64),
            "g": np.full_like(nuc, g), "kappa": kappa}


def disk_albedo(lam_um):
    return 0.5 * np.exp(-np.asarray(lam_um) / 10.0)


def chi_at_1um(beta_albedo="config0"):
    """extinction at exactly 1 um of the continuous dust laws"""
    if beta_albedo == "config0":
        return 100.0 / (1.0 - 0.5)
    return 100.0 / (1.0 - float(disk_albedo(1.0)))


def _grid(n, half_width):
    return {"n": [int(n)] * 3, "lo": [-half_width] * 3, "hi": [half_width] * 3}


def _cell_subsamples(n, lo, hi, sub):
    """coordinates of sub^3 mid-point sub-samples of every cell along one axis"""
    dx = (hi - lo) / n
    off = (np.arange(sub) + 0.5) / sub
    return lo + (np.arange(n)[:, None] + off[None, :]) * dx  # (n, sub)


def sphere_density(n, half_width, radius, rho0, sub=4):
    """uniform sphere averaged over sub^3 mid-point samples per cell"""
    xs = _cell_subsamples(n, -half_width, half_width, sub)  # (n, sub)
    rho = np.zeros((n, n, n))
    x2 = xs ** 2
    for kz in range(n):
        z2 = x2[kz]  # (sub,)
        # broadcast over (iy, ix, sy, sx, sz)
        r2 = (x2[None, :, None, :, None] + x2[:, None, :, None, None] + z2[None, None, None, None, :])
        frac = (r2 < radius * radius).mean(axis=(2, 3, 4))  # (iy, ix)
        rho[kz] = rho0 * frac
    return rho  # indexed [k, j, i] -> C order with x fastest


def config0(n=32, tau=1.0, n_packets=100000, n_iter=5, seed=1, n_bins=100, images=False,
            g=0.6, albedo=0.5, beta=1.0, teff=5800.0, lum=1.0 * L_SUN, half_width=1.0 * AU,
            radius=0.9 * AU):
    nu = nu_edges_log(n_bins)
    dust = powerlaw_dust(nu, beta, albedo=albedo, g=g)
    chi1 = 100.0 / (1.0 - albedo)
    rho0 = tau / (chi1 * radius)
    rho = sphere_density(n, half_width, radius, rho0)
    obs = {"n_incl": 10}
    if images:
        obs.update({"img_npix": 64, "img_half_width": half_width,
                    "img_nu_bins": [bin_of_wavelength(nu, l) for l in (1.0, 10.0, 100.0)]})
    return {
        "name": f"sphere{n}",
        "grid": _grid(n, half_width),
        "rho": rho,
        "nu_edges": nu,
        "dust": dust,
        "sources": [{"pos": [0.0, 0.0, 0.0], "lum": lum, "teff": teff}],
        "observers": obs,
        "run": {"n_packets": int(n_packets), "n_packets_final": int(n_packets), "n_iter": n_iter,
                "seed": seed, "t_init": 10.0},
        "meta": {"rho0": rho0, "tau_1um": tau, "radius": radius, "beta": beta},
    }


def disk_density(n, half_width, rho0, r_in=1.0 * AU, r_out=100.0 * AU, sub=4):
    """flared disk; mid-point sub-samples in x and y, exact Gaussian integral in z"""
    from scipy.special import erf

    dx = 2.0 * half_width / n
    xs = _cell_subsamples(n, -half_width, half_width, sub).ravel()  # (n*sub,)
    X, Y = np.meshgrid(xs, xs, indexing="xy")  # (n*sub [y], n*sub [x])
    R = np.sqrt(X * X + Y * Y)
    inside = (R >= r_in) & (R <= r_out)
    Rs = np.where(inside, R, r_in)
    h = 0.05 * Rs * (Rs / AU) ** 0.125
    surf = np.where(inside, rho0 * (Rs / AU) ** -1.0, 0.0)
    zw = -half_width + np.arange(n + 1) * dx
    rho = np.zeros((n, n, n))
    s2h = math.sqrt(2.0) * h
    prev = erf(zw[0] / s2h)
    for kz in range(n):
        cur = erf(zw[kz + 1] / s2h)
        avg = surf * h * math.sqrt(math.pi / 2.0) * (cur - prev) / dx  # mean over the z extent
        prev = cur
        rho[kz] = avg.reshape(n, sub, n, sub).mean(axis=(1, 3))
    return rho


def config1(n=128, n_packets=10_000_000, n_iter=10, seed=2, n_bins=200, tau=1e3,
            teff=4000.0, rstar=2.0 * R_SUN, npix=256, g=0.6, half_width=120.0 * AU):
    nu = nu_edges_log(n_bins)
    dust = powerlaw_dust(nu, 1.5, g=g, albedo_fn=disk_albedo)
    chi1 = chi_at_1um("disk")
    rho0 = tau / (chi1 * AU * math.log(100.0))
    rho = disk_density(n, half_width, rho0)
    lum = 4.0 * math.pi * rstar ** 2 * SIGMA_SB * teff ** 4
    return {
        "name": f"disk{n}",
        "grid": _grid(n, half_width),
        "rho": rho,
        "nu_edges": nu,
        "dust": dust,
        "sources": [{"pos": [0.0, 0.0, 0.0], "lum": lum, "teff": teff}],
        "observers": {"n_incl": 10, "img_npix": npix, "img_half_width": half_width,
                      "img_nu_bins": [bin_of_wavelength(nu, l) for l in (1.0, 10.0, 100.0)]},
        "run": {"n_packets": int(n_packets), "n_packets_final": int(n_packets), "n_iter": n_iter,
                "seed": seed, "t_init": 10.0},
        "meta": {"rho0": rho0, "tau_1um": tau},
    }


def gaussian_random_field(n, slope=-11.0 / 3.0, seed=1002):
    """unit-variance periodic Gaussian field with power spectrum k^slope (k=0 removed)"""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    f = np.fft.rfftn(white)
    kx = np.fft.fftfreq(n)
    kz = np.fft.rfftfreq(n)
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (slope / 4.0)  # sqrt(P) = k^(slope/2)
    f *= amp
    del white
    g = np.fft.irfftn(f, s=(n, n, n))
    g -= g.mean()
    g /= g.std()
    return g


def clump_sources(n, n_src, rng, half_width, l_min=0.1, l_max=1e3, t_min=3000.0, t_max=20000.0):
    cells = rng.choice(n ** 3, size=n_src, replace=False)
    dx = 2.0 * half_width / n
    k, j, i = np.unravel_index(cells, (n, n, n))
    u = rng.random(n_src)
    a, b = l_min ** -0.5, l_max ** -0.5
    lum = (a - u * (a - b)) ** -2.0 * L_SUN  # inverse CDF of dN/dL ~ L^-1.5
    teff = np.exp(rng.uniform(math.log(t_min), math.log(t_max), n_src))
    src = []
    for s in range(n_src):
        pos = [-half_width + (i[s] + 0.5) * dx, -half_width + (j[s] + 0.5) * dx,
               -half_width + (k[s] + 0.5) * dx]
        src.append({"pos": pos, "lum": float(lum[s]), "teff": float(teff[s])})
    return src


def config2(n=256, n_packets=100_000_000, n_iter=8, seed=3, gen_seed=1002, n_bins=200,
            n_src=50, tau_mean=50.0, sigma_ln=1.5, box=0.65 * PC):
    nu = nu_edges_log(n_bins)
    dust = powerlaw_dust(nu, 1.5, albedo_fn=disk_albedo)
    chi1 = chi_at_1um("disk")
    rho_mean = tau_mean / (chi1 * box)
    g = gaussian_random_field(n, seed=gen_seed)
    lr = sigma_ln * g
    rho = np.exp(lr - lr.max())
    rho *= rho_mean / rho.mean()
    del g, lr
    rng = np.random.default_rng(gen_seed + 1)
    half = 0.5 * box
    return {
        "name": f"clump{n}",
        "grid": _grid(n, half),
        "rho": rho,
        "nu_edges": nu,
        "dust": dust,
        "sources": clump_sources(n, n_src, rng, half),
        "observers": {"n_incl": 10},
        "run": {"n_packets": int(n_packets), "n_packets_final": int(n_packets), "n_iter": n_iter,
                "seed": seed, "t_init": 10.0},
        "meta": {"rho_mean": rho_mean, "tau_mean": tau_mean},
    }


def config3_model(m, packets_per_cell=30, n_iter=5, n_min=16, n_max=96):
    """member m of the batched family: a config-0 sphere or a config-1 disk"""
    rng = np.random.default_rng(3000 + m)
    n = int(rng.integers(n_min, n_max + 1))
    family = "sphere" if rng.random() < 0.5 else "disk"
    tau = 10.0 ** rng.uniform(-1.0, 3.0)
    teff = float(rng.uniform(3000.0, 10000.0))
    g = float(rng.uniform(0.0, 0.8))
    npk = packets_per_cell * n ** 3
    if family == "sphere":
        cfg = config0(n=n, tau=tau, n_packets=npk, n_iter=n_iter, seed=3000 + m, g=g, teff=teff)
    else:
        cfg = config1(n=n, tau=tau, n_packets=npk, n_iter=n_iter, seed=3000 + m, teff=teff, g=g,
                      npix=1)
        cfg["observers"] = {"n_incl": 10}
    cfg["name"] = f"batch{m}-{family}{n}"
    cfg["meta"].update({"family": family, "model": m})
    return cfg


def slab(n=20, tau_1um=1.0, n_packets=200000, seed=7, n_bins=8):
    """pure absorber (albedo 0) filling exactly the cells with 0.2 < z < 0.4
    of a 20^3 grid over [-1, 1]^3 AU; flat source spectrum over the bins"""
    half = 1.0 * AU
    nu = nu_edges_log(n_bins, 0.3, 30.0)
    nuc = bin_centres(nu)
    kappa = 100.0 * (nuc / (C_LIGHT / MICRON)) ** 1.0
    dust = {"chi": kappa.copy(), "albedo": np.zeros(n_bins), "g": np.zeros(n_bins), "kappa": kappa}
    thick = 0.2 * AU
    rho0 = tau_1um / (100.0 * thick)
    rho = np.zeros((n, n, n))
    rho[12:14, :, :] = rho0  # z cells 12, 13 span [0.2, 0.4] AU
    return {
        "name": "slab",
        "grid": _grid(n, half),
        "rho": rho,
        "nu_edges": nu,
        "dust": dust,
        "sources": [{"pos": [0.0, 0.0, 0.0], "lum": L_SUN, "spectrum": np.ones(n_bins)}],
        "observers": {"n_incl": 10},
        "run": {"n_packets": int(n_packets), "n_packets_final": int(n_packets), "n_iter": 1,
                "seed": seed, "t_init": 10.0},
        "meta": {"rho0": rho0, "thickness": thick, "z0": 0.2 * AU},
    }


def clump_config4(n=128, seed=45000, n_src=50, n_packets=None, n_iter=30):
    """unseen test clump for the learned warm start: built like config2"""
    cfg = config2(n=n, gen_seed=seed, n_src=n_src, n_packets=n_packets or 12_500_000,
                  n_iter=n_iter, seed=seed)
    cfg["name"] = f"clump{n}-{seed}"
    return cfg
