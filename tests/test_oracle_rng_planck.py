"""Pins of the oracle's building blocks: Philox4x32-10 and Planck integrals.

Philox is pinned by the published known-answer vectors; the uniforms by
their moments; the Planck bin integrals by independent quadrature and the
closed forms int_0^inf x^3/(e^x-1) dx = pi^4/15 and int B_nu dnu = sigma T^4/pi.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

HERE = os.path.dirname(os.path.abspath(__file__))

H = 6.62607015e-27
K = 1.380649e-16
C = 2.99792458e10
SIGMA = 2 * math.pi ** 5 * K ** 4 / (15 * H ** 3 * C ** 2)


def load_kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = load_kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(orc.philox(ctr, key)) == out


def test_uniform_moments_and_range(orc):
    u = orc.uniform_block(1, 0, 0, 20000, 10).ravel()
    assert u.min() > 0.0 and u.max() < 1.0
    n = u.size
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 4 * math.sqrt(1 / 180 / n)
    # equidistribution over 100 cells (chi-square, 99 dof)
    h, _ = np.histogram(u, bins=100, range=(0, 1))
    chi2 = ((h - n / 100) ** 2 / (n / 100)).sum()
    assert chi2 < 99 + 5 * math.sqrt(2 * 99)
    # consecutive draws and neighbouring packets are uncorrelated
    a = orc.uniform_block(1, 0, 0, 20000, 2)
    r = np.corrcoef(a[:, 0], a[:, 1])[0, 1]
    assert abs(r) < 4 / math.sqrt(20000)
    r2 = np.corrcoef(a[:-1, 0], a[1:, 0])[0, 1]
    assert abs(r2) < 4 / math.sqrt(20000)


def test_uniform_keyed_by_iteration_and_seed(orc):
    a = orc.uniform_block(1, 0, 0, 100, 4)
    b = orc.uniform_block(1, 1, 0, 100, 4)
    c = orc.uniform_block(2, 0, 0, 100, 4)
    assert not np.any(a == b) and not np.any(a == c)
    # packet p of a block starting at p0 is the same stream as in a block starting at 0
    d = orc.uniform_block(1, 0, 37, 10, 4)
    assert np.array_equal(d, a[37:47])


def test_planck_total_is_pi4_over_15(orc):
    assert orc.planck_x_integral(0.0, math.inf) == pytest.approx(math.pi ** 4 / 15, rel=1e-14)
    # contiguous bins add up to the whole
    edges = np.concatenate([[0.0], np.logspace(-6, math.log10(700.0), 301), [math.inf]])
    s = sum(orc.planck_x_integral(a, b) for a, b in zip(edges[:-1], edges[1:]))
    assert s == pytest.approx(math.pi ** 4 / 15, rel=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_planck_bins_vs_quadrature(orc, seed):
    rng = np.random.default_rng(seed)
    f = lambda x: x ** 3 / math.expm1(x) if x > 0 else 0.0
    for _ in range(40):
        a = 10 ** rng.uniform(-4, 1.8)
        b = a * 10 ** rng.uniform(0.001, 1.0)
        ref, err = integrate.quad(f, a, b, epsabs=0, epsrel=1e-13, limit=200)
        assert orc.planck_x_integral(a, b) == pytest.approx(ref, rel=1e-11, abs=1e-300)
    # intervals straddling the series switch
    for a, b in [(1.0, 2.0), (1.4999, 1.5001), (0.01, 30.0), (1.5, 1.6)]:
        ref, _ = integrate.quad(f, a, b, epsabs=0, epsrel=1e-13, limit=200)
        assert orc.planck_x_integral(a, b) == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("T", [3.0, 40.0, 600.0, 5800.0, 20000.0])
def test_planck_bin_integrates_to_sigma_T4_over_pi(orc, T):
    tot = orc.planck_bin(1e-3 * K * T / H, 2e3 * K * T / H, T)
    assert tot == pytest.approx(SIGMA * T ** 4 / math.pi, rel=1e-9)


def test_planck_bin_narrow_bin_matches_B_nu(orc):
    T = 300.0
    for nu in [1e11, 1e12, 1e13, 1e14]:
        dnu = 1e-4 * nu
        bnu = 2 * H * nu ** 3 / C ** 2 / math.expm1(H * nu / (K * T))
        assert orc.planck_bin(nu - dnu / 2, nu + dnu / 2, T) == pytest.approx(bnu * dnu, rel=1e-7)
