"""Pins of the oracle's raytracing of source and dust emission (Sec. 2.6.3).

The expected values are written independently of the oracle's code: the bin
Planck integral by scipy quadrature of B_nu, chords through boxes by a slab
intersection in numpy.

* A uniform cube at one temperature seen along an axis: every pixel's ray
  crosses the full side L, I_k = S_k (1 - exp(-rho chi_k L)) with
  S_k = kappa_k / chi_k B_k(T).
* Two slabs along the line of sight: the far slab's emission is attenuated by
  the near one, I = S_near (1 - e^-tau_near) + e^-tau_near S_far (1 - e^-tau_far)
  (front-to-back order; swapping near and far fails).
* Oblique views of a uniform cube and of a cube filled on one side only: each
  pixel's I = S (1 - exp(-rho chi l)) with l the chord through the filled part.
* Point sources: with no dust L_k/(4 pi) exactly, in the pixel of their
  projection; through a grey cube L/(4 pi) exp(-rho chi s).
* Against the method's other estimator of the same light: with albedo 0 the
  peeled re-emission (component 1) of a final pass estimates the raytraced
  dust SED, and the peeled source light (component 0) the raytraced sources.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from paper_1112_1071_amd import synth

H = 6.62607015e-27
K_B = 1.380649e-16
C_L = 2.99792458e10


def planck_bin(nu_lo, nu_hi, T):
    """int B_nu(T) d nu over the bin, erg/s/cm^2/sr, by adaptive quadrature."""
    x_lo, x_hi = H * nu_lo / (K_B * T), H * nu_hi / (K_B * T)
    if x_lo > 700.0:  # below 1e-290 of the peak
        return 0.0
    f = lambda x: x ** 3 / math.expm1(x) if 0 < x < 700.0 else 0.0  # noqa: E731
    val, _ = quad(f, x_lo, min(x_hi, 700.0), epsabs=0.0, epsrel=1e-12, limit=200)
    return 2.0 * (K_B * T) ** 4 / (H ** 3 * C_L ** 2) * val


def _dust(cfg, chi, albedo):
    n = len(cfg["nu_edges"]) - 1
    cfg["dust"] = {"chi": np.asarray(chi, float) * np.ones(n), "albedo": np.asarray(albedo, float) * np.ones(n),
                   "g": np.zeros(n)}
    return cfg


def _model(cfg, T, dirs):
    cfg["peeloff"] = {"dirs": dirs}
    m = oracle.OracleModel(cfg)
    m.set_temperature(np.broadcast_to(np.asarray(T, float), (np.asarray(cfg["rho"]).size,)).copy())
    return m


def _source_function(cfg, T):
    nu = cfg["nu_edges"]
    d = cfg["dust"]
    kap = d["chi"] * (1.0 - d["albedo"])
    return np.array([kap[k] / d["chi"][k] * planck_bin(nu[k], nu[k + 1], T) for k in range(len(nu) - 1)])


def _dust_pixels(cfg, npix, hw, o):
    """mask of the pixels without the point source (whose pixel also holds its
    light, sed[:, 0])"""
    cen = 0.5 * (np.asarray(cfg["grid"]["lo"], float) + np.asarray(cfg["grid"]["hi"], float))
    o = np.asarray(o, float)
    ex = np.array([-o[1], o[0], 0.0])
    en = np.hypot(ex[0], ex[1])
    ex = np.array([1.0, 0.0, 0.0]) if en < 1e-12 else ex / en
    ey = np.cross(o, ex)
    keep = np.ones((npix, npix), bool)
    for s in cfg["sources"]:
        p = np.asarray(s["pos"], float) - cen
        X, Y = p @ ex, p @ ey
        fx, fy = int(math.floor((X + hw) / (2 * hw) * npix)), int(math.floor((Y + hw) / (2 * hw) * npix))
        if 0 <= fx < npix and 0 <= fy < npix:
            keep[fy, fx] = False
    return keep


def _close(a, b, rtol):
    # relative per value, with an absolute floor far below the largest value
    # (the deep Wien tail of a bin holds values near the underflow limit)
    np.testing.assert_allclose(a, b, rtol=rtol, atol=1e-13 * np.max(np.abs(b)))


def _chords(q0, o, lo, hi):
    """chord length of the lines q0 + s o (q0: [..., 3]) through the box [lo, hi]"""
    s0 = np.full(q0.shape[:-1], -np.inf)
    s1 = np.full(q0.shape[:-1], np.inf)
    for a in range(3):
        if o[a] != 0.0:
            u = (lo[a] - q0[..., a]) / o[a]
            v = (hi[a] - q0[..., a]) / o[a]
            s0 = np.maximum(s0, np.minimum(u, v))
            s1 = np.minimum(s1, np.maximum(u, v))
        else:
            out = (q0[..., a] < lo[a]) | (q0[..., a] >= hi[a])
            s1 = np.where(out, -np.inf, s1)
    return np.maximum(s1 - s0, 0.0)


def _pixel_points(o, npix, hw):
    o = np.asarray(o, float)
    ex = np.array([-o[1], o[0], 0.0])
    en = np.hypot(ex[0], ex[1])
    ex = np.array([1.0, 0.0, 0.0]) if en < 1e-12 else ex / en
    ey = np.cross(o, ex)
    c = -hw + (np.arange(npix) + 0.5) * (2 * hw / npix)
    Y, X = np.meshgrid(c, c, indexing="ij")  # [iy][ix]
    return X[..., None] * ex + Y[..., None] * ey


@pytest.mark.parametrize("o", [[0, 0, 1], [-1, 0, 0], [0, 1, 0]])
def test_uniform_cube_along_an_axis(orc, o):
    n, half = 6, synth.AU
    cfg = _dust(synth.config0(n=n, n_packets=10, n_iter=1, n_bins=12), chi=[80.0], albedo=[0.3])
    rho0 = 1.5 / (80.0 * 2 * half)  # tau = 1.5 across the cube
    cfg["rho"][:] = rho0
    T = 45.0
    m = _model(cfg, T, [o])
    npix = 12  # pixel centres a quarter cell from the walls
    sed, cube = m.raytrace(npix, half)
    S = _source_function(cfg, T)
    chi = cfg["dust"]["chi"]
    apix = (2 * half / npix) ** 2
    want = S * -np.expm1(-rho0 * chi * 2 * half) * apix
    keep = _dust_pixels(cfg, npix, half, o)
    _close(cube[0][keep], np.broadcast_to(want, cube[0][keep].shape), 1e-10)
    _close(sed[0, 1], want * npix * npix, 1e-10)


def test_two_slabs_front_to_back(orc):
    half = synth.AU
    cfg = _dust(synth.config0(n=4, n_packets=10, n_iter=1, n_bins=10), chi=[120.0], albedo=[0.0])
    cfg["grid"]["n"] = [4, 4, 2]
    rho = np.zeros((2, 4, 4))
    rho[0] = 2.0 / (120.0 * half)  # z < 0: tau 2 along z
    rho[1] = 0.5 / (120.0 * half)  # z > 0: tau 0.5
    cfg["rho"] = rho
    T = np.zeros((2, 4, 4))
    T[0], T[1] = 30.0, 80.0
    m = _model(cfg, T.reshape(-1), [[0, 0, 1]])  # observer on +z: the z > 0 slab is in front
    npix = 8
    sed, cube = m.raytrace(npix, half)
    S_far, S_near = _source_function(cfg, 30.0), _source_function(cfg, 80.0)
    want = (S_near * -math.expm1(-0.5) + math.exp(-0.5) * S_far * -math.expm1(-2.0)) * (2 * half / npix) ** 2
    keep = _dust_pixels(cfg, npix, half, [0, 0, 1])
    _close(cube[0][keep], np.broadcast_to(want, cube[0][keep].shape), 1e-10)


@pytest.mark.parametrize("o", [[0.48, -0.6, 0.64], [-0.36, 0.48, -0.8], [0.6, 0.8, 0.0]])
def test_oblique_chords(orc, o):
    n, half = 7, synth.AU
    cfg = _dust(synth.config0(n=n, n_packets=10, n_iter=1, n_bins=8), chi=[60.0], albedo=[0.2])
    rho0 = 3.0 / (60.0 * 2 * half)
    cfg["rho"][:] = rho0
    T = 55.0
    m = _model(cfg, T, [o])
    npix, hw = 23, 1.9 * half
    sed, cube = m.raytrace(npix, hw)
    q = _pixel_points(o, npix, hw)
    chord = _chords(q, np.asarray(o, float), np.full(3, -half), np.full(3, half))
    assert (chord > 0).sum() > 100 and (chord == 0).sum() > 10
    S = _source_function(cfg, T)
    chi = cfg["dust"]["chi"]
    want = S[None, None, :] * -np.expm1(-rho0 * chi[None, None, :] * chord[..., None]) * (2 * hw / npix) ** 2
    keep = _dust_pixels(cfg, npix, hw, o)
    _close(cube[0][keep], want[keep], 1e-9)


@pytest.mark.parametrize("o", [[0.48, -0.6, 0.64], [-0.8, 0.0, 0.6]])
def test_half_filled_cube(orc, o):
    # only the cells with x < 0 hold dust: each ray's optical depth comes from
    # its chord through the half box [-half, 0] x [-half, half]^2
    n, half = 8, synth.AU
    cfg = _dust(synth.config0(n=n, n_packets=10, n_iter=1, n_bins=6), chi=[90.0], albedo=[0.4])
    rho0 = 2.5 / (90.0 * half)
    rho = np.zeros((n, n, n))
    rho[:, :, : n // 2] = rho0
    cfg["rho"] = rho
    T = 70.0
    m = _model(cfg, T, [o])
    npix, hw = 21, 1.8 * half
    sed, cube = m.raytrace(npix, hw)
    q = _pixel_points(o, npix, hw)
    chord = _chords(q, np.asarray(o, float), np.array([-half, -half, -half]), np.array([0.0, half, half]))
    assert (chord > 0).sum() > 50
    S = _source_function(cfg, T)
    chi = cfg["dust"]["chi"]
    want = S[None, None, :] * -np.expm1(-rho0 * chi[None, None, :] * chord[..., None]) * (2 * hw / npix) ** 2
    keep = _dust_pixels(cfg, npix, hw, o)
    _close(cube[0][keep], want[keep], 1e-9)


def test_sources_without_dust_and_through_a_grey_cube(orc):
    half = synth.AU
    cfg = synth.config0(n=6, n_packets=10, n_iter=1, n_bins=15)
    cfg["rho"][:] = 0.0
    cfg["sources"] = [{"pos": [0.2 * half, -0.3 * half, 0.1 * half], "lum": synth.L_SUN, "teff": 5000.0},
                      {"pos": [-0.5 * half, 0.4 * half, -0.6 * half], "lum": 3 * synth.L_SUN, "teff": 9000.0}]
    dirs = [[0, 0, 1], [0.6, 0, 0.8]]
    m = _model(cfg, 20.0, dirs)
    sed, cube = m.raytrace(10, 1.2 * half)
    nu = cfg["nu_edges"]
    want = np.zeros(len(nu) - 1)
    for s in cfg["sources"]:
        lb = np.array([planck_bin(nu[k], nu[k + 1], s["teff"]) for k in range(len(nu) - 1)])
        want += s["lum"] * lb / lb.sum() / (4 * math.pi)
    for i in range(2):
        np.testing.assert_allclose(sed[i, 0], want, rtol=1e-9)
        assert not np.any(sed[i, 1])
        np.testing.assert_allclose(cube[i].sum(axis=(0, 1)), want, rtol=1e-9)
        assert np.count_nonzero(cube[i].sum(axis=2)) == 2  # two source pixels
    # grey cube, source at the centre, along axes and a diagonal-ish direction
    cfg = _dust(synth.config0(n=8, n_packets=10, n_iter=1, n_bins=5), chi=[150.0], albedo=[0.5])
    rho0 = 2.0 / (150.0 * half)
    cfg["rho"][:] = rho0
    dirs = [[0, 0, 1], [0.6, 0, 0.8], [0.48, -0.6, 0.64]]
    m = _model(cfg, 20.0, dirs)
    sed, _ = m.raytrace(8, half)
    for i, dist in enumerate([1.0, 1.25, 1.0 / 0.64]):
        assert sed[i, 0].sum() == pytest.approx(synth.L_SUN / (4 * math.pi) * math.exp(-2.0 * dist), rel=1e-10)


def test_raytrace_matches_peeled_emission(orc):
    # albedo 0: the final pass's peeled re-emission estimates the dust emission
    # at the temperatures it re-emits with, the peeled source light the
    # attenuated sources; both per steradian, the same as the raytraced SED
    # (an optically thin sphere, so that emission inside a cell is uniform).
    # The raytraced SED is the sum over pixels, one ray per pixel centre: a
    # quadrature of the image plane that converges when every cell projects
    # onto many pixels -- oblique views here; along a grid axis each pixel
    # samples one column of cells and the few hot columns at the source alias.
    cfg = synth.config0(n=20, tau=1.0, n_packets=400000, n_iter=4, n_bins=30, albedo=0.0)
    dirs = [[0.48, -0.6, 0.64], [-0.36, 0.48, -0.8]]
    cfg["peeloff"] = {"dirs": dirs}
    m = oracle.OracleModel(cfg)
    for _ in range(4):
        m.iterate()
    m.final_pass()
    ps, ps2 = m.peeled_sed()
    sed, _ = m.raytrace(128, 1.05 * math.sqrt(3) * synth.AU)
    for i in range(2):
        for comp in (0, 1):
            ok = ps[i, comp] > 0.02 * ps[i, comp].max()
            assert ok.sum() >= 8
            z = (ps[i, comp][ok] - sed[i, comp][ok]) / np.sqrt(ps2[i, comp][ok])
            assert np.mean(np.abs(z) < 4) >= 0.9, (i, comp, z)
            tot = (ps[i, comp].sum() - sed[i, comp].sum()) / math.sqrt(ps2[i, comp].sum())
            assert abs(tot) < 4, (i, comp, tot)
