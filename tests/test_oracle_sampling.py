"""Pins of the oracle's direction sampling: isotropic moments (a closed form
named for this method), Henyey-Greenstein moments and cumulative
distribution, and the direction rotation."""
import math

import numpy as np
import pytest


def test_isotropic_moments(orc):
    u = orc.uniform_block(5, 0, 0, 100000, 2)
    d = np.array([orc.isotropic(a, b) for a, b in u])
    n = len(d)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)
    # <d> = 0 (var of each component 1/3)
    assert np.all(np.abs(d.mean(axis=0)) < 4 * math.sqrt(1 / 3 / n))
    # <d_a d_b> = delta_ab / 3 ; var(d_a^2) = 1/5 - 1/9, var(d_a d_b) = 1/15
    M = d.T @ d / n
    for a in range(3):
        assert abs(M[a, a] - 1 / 3) < 4 * math.sqrt((1 / 5 - 1 / 9) / n)
        for b in range(a + 1, 3):
            assert abs(M[a, b]) < 4 * math.sqrt(1 / 15 / n)


def test_isotropic_special_values(orc):
    assert np.allclose(orc.isotropic(1.0, 0.0), [0, 0, 1])
    assert np.allclose(orc.isotropic(0.0, 0.0), [0, 0, -1])
    assert np.allclose(orc.isotropic(0.5, 0.25), [0, 1, 0], atol=1e-15)


@pytest.mark.parametrize("g", [0.0, 0.3, 0.6, 0.9, -0.5])
def test_hg_moments(orc, g):
    n = 200001
    u = (np.arange(n) + 0.5) / n
    mu = np.array([orc.hg_mu(g, x) for x in u])
    assert mu.min() >= -1 and mu.max() <= 1
    assert mu.mean() == pytest.approx(g, abs=2e-6)
    assert (mu ** 2).mean() == pytest.approx((1 + 2 * g * g) / 3, abs=2e-6)


@pytest.mark.parametrize("g", [0.2, 0.6, 0.95, -0.7])
def test_hg_inverse_cdf(orc, g):
    # P(mu' <= mu) for p(mu) = (1-g^2)/2 (1+g^2-2 g mu)^(-3/2)
    def cdf(mu):
        return (1 - g * g) / (2 * g) * ((1 + g * g - 2 * g * mu) ** -0.5 - 1 / (1 + g))

    for u in np.linspace(0.001, 0.999, 57):
        assert cdf(orc.hg_mu(g, u)) == pytest.approx(u, abs=1e-12)


def test_hg_g0_is_isotropic(orc):
    for u in [0.0, 0.1, 0.5, 0.77, 1.0]:
        assert orc.hg_mu(0.0, u) == pytest.approx(2 * u - 1, abs=1e-15)


def test_rotate_angle_and_norm(orc):
    rng = np.random.default_rng(3)
    for _ in range(500):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        mu = rng.uniform(-1, 1)
        phi = rng.uniform(0, 2 * math.pi)
        o = orc.rotate(d, mu, phi)
        assert np.linalg.norm(o) == pytest.approx(1.0, abs=1e-14)
        assert o @ d == pytest.approx(mu, abs=1e-12)
    d = np.array([0.0, 0.0, 1.0])
    assert np.allclose(orc.rotate(d, 1.0, 0.3), d)
    assert np.allclose(orc.rotate(d, -1.0, 0.3), -d)


def test_rotate_azimuth_uniform_around_axis(orc):
    # for fixed d and mu, the new direction's component perpendicular to d has
    # zero mean when phi is uniform
    d = np.array([0.3, -0.4, math.sqrt(1 - 0.25)])
    phis = (np.arange(4096) + 0.5) / 4096 * 2 * math.pi
    o = np.array([orc.rotate(d, 0.2, p) for p in phis])
    assert np.allclose(o.mean(axis=0), 0.2 * d, atol=1e-12)


def test_rotate_pole_branch_continuous(orc):
    # the near-pole branch agrees with the general formula just outside it
    eps = 1e-9
    d1 = np.array([math.sqrt(1 - (1 - eps) ** 2), 0.0, 1 - eps])
    o1 = orc.rotate(d1, 0.3, 1.1)
    d0 = np.array([0.0, 0.0, 1.0])
    o0 = orc.rotate(d0, 0.3, 1.1)
    # both at angle acos(0.3) from their axes, and the axes differ by ~sqrt(2 eps)
    assert o1 @ d1 == pytest.approx(0.3, abs=1e-9)
    assert o0 @ d0 == pytest.approx(0.3, abs=1e-12)
