"""Pins of the oracle's peeling-off (Sec. 2.6.2).

* No dust: every source packet peels eps/(4 pi) unattenuated, so the peeled
  SED of every observer sums to L/(4 pi) exactly, with no processed part.
* Grey dust, source at the centre of a uniform cube: the direct component is
  L/(4 pi) exp(-rho chi s), s the distance to the cube's surface along the
  observer direction, exactly (each packet's direct peel is deterministic).
* A spherically symmetric model: the peeled SED (per steradian) estimates the
  same escaping flux as the binned SED of the inclination bin holding the
  observer (binned energy / (4 pi / n_incl)); z-test per frequency bin.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1112_1071_amd import synth


def _grey(cfg, chi=150.0, albedo=0.5, g=0.6):
    n = len(cfg["nu_edges"]) - 1
    cfg["dust"] = {"chi": np.full(n, chi), "albedo": np.full(n, albedo), "g": np.full(n, g)}
    return cfg


def test_peeloff_no_dust_is_exact(orc):
    cfg = synth.config0(n=16, n_packets=20000, n_iter=1)
    cfg["rho"][:] = 0.0
    dirs = [[0, 0, 1], [1, 0, 0], [0.6, 0, 0.8], [0, -0.28, -0.96]]
    cfg["peeloff"] = {"dirs": dirs}
    o = oracle.OracleModel(cfg)
    o.final_pass()
    s, _ = o.peeled_sed()
    np.testing.assert_allclose(s[:, 0].sum(axis=1), synth.L_SUN / (4 * math.pi), rtol=1e-12)
    assert not np.any(s[:, 1])


@pytest.mark.parametrize("o,dist", [([0, 0, 1], 1.0), ([-1, 0, 0], 1.0), ([0.6, 0, 0.8], 1.25),
                                    ([0.48, -0.6, 0.64], 1.0 / 0.64)])
def test_peeloff_direct_attenuation_grey_cube(orc, o, dist):
    n, half = 12, synth.AU
    cfg = _grey(synth.config0(n=n, n_packets=5000, n_iter=1))
    rho0 = 2.0 / (150.0 * half)  # tau = 2 from the centre to a face
    cfg["rho"][:] = rho0
    cfg["peeloff"] = {"dirs": [o]}
    m = oracle.OracleModel(cfg)
    m.final_pass()
    s, _ = m.peeled_sed()
    want = synth.L_SUN / (4 * math.pi) * math.exp(-rho0 * 150.0 * dist * half)
    assert s[0, 0].sum() == pytest.approx(want, rel=1e-10)
    assert s[0, 1].sum() > 0


def test_peeloff_matches_binning_for_a_sphere(orc):
    n_incl = 10
    cfg = synth.config0(n=24, tau=1.0, n_packets=300000, n_iter=1, n_bins=20)
    # observer directions inside inclination bins 2 and 7 (|d_z| in [0.2,0.3), [0.7,0.8))
    dirs = []
    for mu in (0.25, 0.75):
        st = math.sqrt(1 - mu * mu)
        dirs.append([st * math.cos(0.3), st * math.sin(0.3), mu])
    cfg["peeloff"] = {"dirs": dirs}
    m = oracle.OracleModel(cfg)
    m.iterate()
    m.final_pass()
    ps, ps2 = m.peeled_sed()
    bs, bs2, bn = m.sed()
    for i, b in enumerate((2, 7)):
        peel = ps[i].sum(axis=0)
        pvar = ps2[i].sum(axis=0)
        binned = bs[b] * n_incl / (4 * math.pi)
        bvar = bs2[b] * (n_incl / (4 * math.pi)) ** 2
        ok = bn[b] >= 30
        assert ok.sum() >= 10
        z = (peel[ok] - binned[ok]) / np.sqrt(pvar[ok] + bvar[ok])
        assert np.mean(np.abs(z) < 4) >= 0.9, z
        tot = (peel.sum() - binned.sum()) / math.sqrt(pvar.sum() + bvar.sum())
        assert abs(tot) < 4, tot
