"""Closed-form pins of the oracle's end-to-end transport.

* exp(-tau) transmission through a pure absorbing slab (per direction and
  frequency bin) and out of a single cubic cell;
* the optically thin limit: each cell's Ȧ equals the cell average of
  (L/4 pi r^2) sum_k p_k kappa_k e^{-tau_k(r)}, and T follows
  T = T_*(R_*/2r)^(2/(4+beta)) with slope -2/(4+beta) in log-log;
* re-emission frequencies follow kappa_nu B_nu of the cell's emission rows.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_1112_1071_amd import synth

H = 6.62607015e-27
K = 1.380649e-16
C = 2.99792458e10
SIGMA = 2 * math.pi ** 5 * K ** 4 / (15 * H ** 3 * C ** 2)


def direct_escapes(m, n):
    ev, cnt = m.event_log()
    direct = (cnt == 2) & (ev[:, 1]["type"] == oracle.EV_ESCAPE)
    return ev, cnt, direct


def test_slab_transmission():
    cfg = synth.slab(n_packets=200000)
    n = cfg["run"]["n_packets"]
    m = oracle.OracleModel(cfg, event_log_packets=n, event_log_cap=2)
    m.iterate()
    ev, cnt, direct = direct_escapes(m, n)
    nu_emit = ev[:, 0]["nu"]
    incl = ev[:, 1]["incl"]
    kappa = cfg["dust"]["chi"]
    rho0 = cfg["meta"]["rho0"]
    thick = cfg["meta"]["thickness"]
    checked = 0
    for k in range(len(kappa)):
        nk = int((nu_emit == k).sum())
        tau = kappa[k] * rho0 * thick
        for b in range(4, 10):
            a, c = b / 10, (b + 1) / 10
            up, _ = integrate.quad(lambda mu: 0.5 * math.exp(-tau / mu), a, c, epsrel=1e-12)
            p = 0.5 * (c - a) + up
            x = int(((nu_emit == k) & direct & (incl == b)).sum())
            z = (x - nk * p) / math.sqrt(nk * p * (1 - p))
            assert abs(z) < 4.5, (k, b, z)
            checked += 1
    assert checked == 48


def test_single_cell_escape_probability():
    # one cubic cell of side 2 with the source at its centre: the probability of
    # leaving without interaction is the sphere average of exp(-tau0 s(Omega)),
    # s = 1/max|d_a| the distance to the surface
    tau0 = 0.7
    cfg = {
        "grid": {"n": [1, 1, 1], "lo": [-1.0] * 3, "hi": [1.0] * 3},
        "rho": np.array([tau0]),
        "nu_edges": np.array([1e13, 2e13]),
        "dust": {"chi": np.array([1.0]), "albedo": np.array([0.0]), "g": np.array([0.0])},
        "sources": [{"pos": [0.0, 0.0, 0.0], "lum": 1.0, "spectrum": np.array([1.0])}],
        "observers": {"n_incl": 10},
        "run": {"n_packets": 100000, "seed": 3},
    }
    n = 100000
    m = oracle.OracleModel(cfg, event_log_packets=n, event_log_cap=2)
    m.iterate()
    _, _, direct = direct_escapes(m, n)

    # sphere average by a fine mid-point rule in (mu, phi)
    nq = 2000
    mu = (np.arange(nq) + 0.5) / nq * 2 - 1
    phi = (np.arange(2 * nq) + 0.5) / (2 * nq) * 2 * math.pi
    M, P = np.meshgrid(mu, phi, indexing="ij")
    S = np.sqrt(1 - M * M)
    dmax = np.maximum(np.maximum(np.abs(S * np.cos(P)), np.abs(S * np.sin(P))), np.abs(M))
    p = float(np.exp(-tau0 / dmax).mean())
    x = direct.sum()
    z = (x - n * p) / math.sqrt(n * p * (1 - p))
    assert abs(z) < 4, (x / n, p)


@pytest.fixture(scope="module")
def thin_run():
    cfg = synth.config0(tau=1e-3, n_packets=2_000_000, n_iter=1)
    m = oracle.OracleModel(cfg, want_noise=1)
    st = m.iterate()
    adot, sig = m.specific_energy(with_sigma=True)
    return cfg, m, st, adot, sig, m.temperature()


def cell_geometry(cfg):
    n = cfg["grid"]["n"][0]
    hw = cfg["grid"]["hi"][0]
    dx = 2 * hw / n
    c = -hw + (np.arange(n) + 0.5) * dx
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel(), dx


def expected_thin_adot(cfg, X, Y, Z, dx, sel):
    """cell average of (L / 4 pi r^2) sum_k p_k kappa_k exp(-rho0 chi_k r), Gauss-Legendre 4^3"""
    nu = cfg["nu_edges"]
    teff = cfg["sources"][0]["teff"]
    L = cfg["sources"][0]["lum"]
    p = np.array([oracle.planck_bin(a, b, teff) for a, b in zip(nu[:-1], nu[1:])])
    p /= p.sum()
    kap = cfg["dust"]["kappa"]
    chi = cfg["dust"]["chi"]
    rho0 = cfg["meta"]["rho0"]
    g, w = np.polynomial.legendre.leggauss(4)
    out = np.zeros(sel.sum())
    xs, ys, zs = X[sel], Y[sel], Z[sel]
    for i, (gx, wx) in enumerate(zip(g, w)):
        for gy, wy in zip(g, w):
            for gz, wz in zip(g, w):
                r = np.sqrt((xs + gx * dx / 2) ** 2 + (ys + gy * dx / 2) ** 2 + (zs + gz * dx / 2) ** 2)
                att = (p[None, :] * kap[None, :] * np.exp(-rho0 * chi[None, :] * r[:, None])).sum(axis=1)
                out += wx * wy * wz / 8 * L / (4 * math.pi * r * r) * att
    return out


def test_thin_limit_specific_energy(thin_run):
    cfg, m, st, adot, sig, T = thin_run
    X, Y, Z, dx = cell_geometry(cfg)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    sel = (r > 3 * dx) & (r + dx < 0.8 * synth.AU)
    E = expected_thin_adot(cfg, X, Y, Z, dx, sel)
    a, s = adot[sel], sig[sel]
    z = (a - E) / s
    assert sel.sum() > 5000
    assert np.mean(np.abs(z) < 4) > 0.995
    assert 0.9 < z.std() < 1.1
    # aggregate: no bias beyond the neglected scattered/re-emitted light (~1e-3)
    ratio = (a / s ** 2).sum() / (E / s ** 2).sum()
    assert ratio == pytest.approx(1.0, abs=2e-3)


def test_thin_limit_temperature_profile(thin_run):
    cfg, m, st, adot, sig, T = thin_run
    X, Y, Z, dx = cell_geometry(cfg)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    sel = (r > 3 * dx) & (r + dx < 0.8 * synth.AU)
    beta = cfg["meta"]["beta"]
    slope = np.polyfit(np.log(r[sel]), np.log(T[sel]), 1)[0]
    assert slope == pytest.approx(-2 / (4 + beta), abs=5e-3)
    # the temperature itself: T = T*(R*/2 r_eff)^(2/(4+beta)) with r_eff^-2 = <r^-2>_cell
    teff = cfg["sources"][0]["teff"]
    L = cfg["sources"][0]["lum"]
    rstar = math.sqrt(L / (4 * math.pi * SIGMA * teff ** 4))
    g, w = np.polynomial.legendre.leggauss(4)
    inv_r2 = np.zeros(sel.sum())
    for gx, wx in zip(g, w):
        for gy, wy in zip(g, w):
            for gz, wz in zip(g, w):
                rr2 = (X[sel] + gx * dx / 2) ** 2 + (Y[sel] + gy * dx / 2) ** 2 + (Z[sel] + gz * dx / 2) ** 2
                inv_r2 += wx * wy * wz / 8 / rr2
    r_eff = inv_r2 ** -0.5
    T_ref = teff * (rstar / (2 * r_eff)) ** (2 / (4 + beta))
    rel = T[sel] / T_ref - 1
    assert abs(np.median(rel)) < 0.01
    assert np.mean(np.abs(rel) < 0.03) > 0.99
    # the paper-scale number: about 674 K at 0.5 AU for this star and beta = 1
    assert teff * (rstar / (2 * 0.5 * synth.AU)) ** 0.4 == pytest.approx(674, abs=2)


def test_reemission_spectrum_follows_rows():
    # a single very opaque pure-absorber cell at a fixed temperature: every
    # re-emission samples kappa_k B_k from row m or m+1 with weight w
    nu = synth.nu_edges_log(30)
    kap = 100 * (synth.bin_centres(nu) / (C / 1e-4))
    T_cell = 287.0
    cfg = {
        "grid": {"n": [1, 1, 1], "lo": [-1.0] * 3, "hi": [1.0] * 3},
        "rho": np.array([5.0]),
        "nu_edges": nu,
        "dust": {"chi": kap, "albedo": np.zeros(30), "g": np.zeros(30)},
        "sources": [{"pos": [0.0, 0.0, 0.0], "lum": 1.0, "teff": 5000.0}],
        "observers": {"n_incl": 10},
        "run": {"n_packets": 4000, "seed": 9},
    }
    m = oracle.OracleModel(cfg, event_log_packets=4000, event_log_cap=4096, max_events=4000)
    m.set_temperature(np.array([T_cell]))
    m.iterate()
    ev, cnt = m.event_log()
    ab = np.concatenate([ev[p, : min(cnt[p], 4096)] for p in range(4000)])
    ab = ab[ab["type"] == oracle.EV_ABSORB]["nu"]
    assert ab.size > 20000
    pos = 127 * math.log(T_cell) / math.log(1e4)
    mrow, w = int(pos), pos - int(pos)
    Tm = [math.exp(math.log(1e4) * r / 127) for r in (mrow, mrow + 1)]

    def row(Tr):
        f = lambda x: x ** 3 / math.expm1(x)
        b = np.array([integrate.quad(f, H * a / (K * Tr), H * c / (K * Tr), epsrel=1e-10)[0]
                      for a, c in zip(nu[:-1], nu[1:])])
        q = kap * b
        return q / q.sum()

    pk = (1 - w) * row(Tm[0]) + w * row(Tm[1])
    h = np.bincount(ab, minlength=30) / ab.size
    big = pk > 1e-3
    z = (h[big] - pk[big]) / np.sqrt(pk[big] * (1 - pk[big]) / ab.size)
    # events of one packet are correlated only through the cell, not the frequency draw
    assert np.all(np.abs(z) < 4.5)
