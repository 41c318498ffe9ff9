"""Pins of the oracle's modified random walk (Sec. 2.2).

* The escape-time sampler inverts F(y) = 1 + 2 sum (-1)^n exp(-n^2 y) (first
  passage of diffusion from the centre of a sphere, y = pi^2 D t / R^2): F is
  re-evaluated here from its series, and the sampled y has the closed-form
  moments E[y] = pi^2/6 and E[y^2] = 7 pi^4/180.
* The step's path length 3 rho chi R^2 y / pi^2 against a brute-force random
  walk of isotropic scatterings (unit mean free path) from the centre of a
  sphere of radius R mean free paths: the same mean (R^2/2) and quantiles, to
  the diffusion approximation's O(1/R) (a wrong factor in D fails).
* Planck- and Rosseland-mean opacities: equal to kappa and chi for grey dust;
  for power-law dust against scipy quadrature of their definitions.
* A thick grey cube around a source: with and without the walk, every packet
  escapes (energy conserved), the walk replaces most interactions, and the
  temperatures agree to the approximation's accuracy.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from paper_1112_1071_amd import synth

H = 6.62607015e-27
K_B = 1.380649e-16


def _F_series(y):
    # valid for y >= 0.3, where the alternating series converges quickly
    n = np.arange(1, 60)
    return 1.0 + 2.0 * np.sum((-1.0) ** n * np.exp(-(n * n) * y))


def test_escape_sampler_inverts_the_series(orc):
    for u in [0.05, 0.2, 0.5, 0.8, 0.99, 0.999999]:
        y = oracle.mrw_escape_y(u)
        assert y > 0.3
        assert _F_series(y) == pytest.approx(u, abs=1e-12)
    # small y (u small): F from the image series 2 sqrt(pi/y) sum exp(-pi^2 (2m+1)^2 / 4y)
    for u in [1e-12, 1e-6, 1e-3]:
        y = oracle.mrw_escape_y(u)
        m = np.arange(0, 20)
        F = 2 * math.sqrt(math.pi / y) * np.sum(np.exp(-(math.pi * (2 * m + 1)) ** 2 / (4 * y)))
        assert F == pytest.approx(u, rel=1e-9)


def test_escape_moments(orc):
    n = 100000
    u = (np.arange(n) + 0.5) / n  # stratified: the mean of y(u) is the integral of the quantile
    y = np.array([oracle.mrw_escape_y(v) for v in u])
    assert y.mean() == pytest.approx(math.pi ** 2 / 6, rel=1e-4)
    assert (y * y).mean() == pytest.approx(7 * math.pi ** 4 / 180, rel=1e-3)


def _random_walk_paths(R, n_walkers, rng):
    """path length until an isotropic scatterer (unit mean free path) started
    at the centre first reaches distance R"""
    x = np.zeros((n_walkers, 3))
    path = np.zeros(n_walkers)
    alive = np.ones(n_walkers, bool)
    while alive.any():
        k = np.flatnonzero(alive)
        mu = 2 * rng.random(k.size) - 1
        phi = 2 * math.pi * rng.random(k.size)
        st = np.sqrt(1 - mu * mu)
        d = np.stack([st * np.cos(phi), st * np.sin(phi), mu], axis=1)
        step = -np.log(rng.random(k.size))
        # distance along d to the sphere |x + s d| = R
        b = np.einsum("ij,ij->i", x[k], d)
        c = np.einsum("ij,ij->i", x[k], x[k]) - R * R
        s_exit = -b + np.sqrt(b * b - c)
        out = step >= s_exit
        path[k] += np.where(out, s_exit, step)
        x[k] += d * np.minimum(step, s_exit)[:, None]
        alive[k[out]] = False
    return path


@pytest.mark.parametrize("R", [10.0, 30.0])
def test_step_length_matches_brute_force_walk(orc, R):
    rng = np.random.default_rng(7)
    rw = _random_walk_paths(R, 6000 if R > 20 else 20000, rng)
    u = (np.arange(20000) + 0.5) / 20000
    mrw = np.array([3.0 * R * R * oracle.mrw_escape_y(v) / math.pi ** 2 for v in u])  # rho chi = 1
    assert mrw.mean() == pytest.approx(R * R / 2, rel=1e-4)
    tol = 2.5 / R  # the diffusion approximation misses O(1/R) (boundary layer of ~1 mean free path)
    assert rw.mean() / mrw.mean() == pytest.approx(1.0, abs=tol)
    for q in (0.1, 0.5, 0.9):
        assert np.quantile(rw, q) / np.quantile(mrw, q) == pytest.approx(1.0, abs=tol + 0.03)


def test_planck_and_rosseland_means(orc):
    cfg = synth.config0(n=4, n_packets=10, n_bins=20)
    n = len(cfg["nu_edges"]) - 1
    cfg["dust"] = {"chi": np.full(n, 70.0), "albedo": np.full(n, 0.4), "g": np.zeros(n)}
    m = oracle.OracleModel(cfg)
    for T in (20.0, 300.0, 3000.0):
        assert m.planck_mean_kappa(T) == pytest.approx(42.0, rel=1e-12)
        assert m.rosseland_chi(T) == pytest.approx(70.0, rel=1e-12)
    m.close()
    cfg = synth.config0(n=4, n_packets=10, n_bins=20)  # power-law dust, albedo 0.5
    m = oracle.OracleModel(cfg)
    nu = cfg["nu_edges"]
    chi = cfg["dust"]["chi"]
    kap = chi * (1 - cfg["dust"]["albedo"])
    for T in (30.0, 500.0):
        def B(x):
            return x ** 3 / math.expm1(x) if 0 < x < 700 else 0.0

        def dB(x):  # x^4 e^x / (e^x - 1)^2 written with e^-x (no overflow)
            return x ** 4 * math.exp(-x) / (-math.expm1(-x)) ** 2 if 0 < x < 700 else 0.0

        xs = H * nu / (K_B * T)
        b = np.array([quad(B, xs[k], xs[k + 1], epsrel=1e-12, limit=200)[0] for k in range(n)])
        db = np.array([quad(dB, xs[k], xs[k + 1], epsrel=1e-12, limit=200)[0] for k in range(n)])
        assert m.planck_mean_kappa(T) == pytest.approx(np.sum(kap * b) / np.sum(b), rel=1e-9)
        assert m.rosseland_chi(T) == pytest.approx(np.sum(db) / np.sum(db / chi), rel=1e-7)
    m.close()


def test_thick_cube_with_and_without_the_walk(orc):
    # grey dust, tau 30 per cell, central source: the walk conserves energy,
    # replaces most interactions, and gives the temperatures of the plain walk
    # to within its Monte-Carlo scatter (measured by a second seed: in cells
    # this thick one packet deposits many times in a cell, so the sum-of-squares
    # error estimate of Eq. 2 undercounts the scatter)
    n, half = 4, synth.AU
    cfg = synth.config0(n=n, n_packets=8000, n_iter=1, n_bins=12)
    nb = len(cfg["nu_edges"]) - 1
    chi = 100.0
    cfg["dust"] = {"chi": np.full(nb, chi), "albedo": np.full(nb, 0.5), "g": np.zeros(nb)}
    cfg["rho"][:] = 30.0 / (chi * 2 * half / n)
    L = sum(s["lum"] for s in cfg["sources"])
    runs = {}
    for gamma, seed in ((0.0, 1), (0.0, 2), (2.0, 1)):
        c = dict(cfg)
        c["run"] = dict(cfg["run"], seed=seed)
        m = oracle.OracleModel(c, mrw_gamma=gamma)
        st = m.iterate()
        assert st["e_escaped"] == pytest.approx(L, rel=1e-12)
        assert st["n_killed"] == 0
        runs[(gamma, seed)] = (st, m.temperature())
        m.close()
    st0, T0 = runs[(0.0, 1)]
    _, T0b = runs[(0.0, 2)]
    st2, T2 = runs[(2.0, 1)]
    assert st0["n_mrw"] == 0 and st2["n_mrw"] > 0
    assert (st2["n_scatter"] + st2["n_absorb"]) * 2 < st0["n_scatter"] + st0["n_absorb"]
    seed_dev = np.abs(T0b / T0 - 1)
    mrw_dev = np.abs(T2 / T0 - 1)
    assert np.median(mrw_dev) <= 1.5 * np.median(seed_dev) + 0.005
    assert np.quantile(mrw_dev, 0.9) <= 1.5 * np.quantile(seed_dev, 0.9) + 0.01
