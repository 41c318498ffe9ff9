"""GPU raytracing of source and dust emission (Sec. 2.6.3) against the FP64
oracle, through the C ABI.

Both sides raytrace the same temperature field (set on both, or the GPU's
own after iterations copied to the oracle).  The GPU integrates the Planck
function over a bin by composite Gauss-Legendre quadrature, the oracle by its
series: they agree to about 1e-12 relative; the ray walks differ only in
rounding.  Bar: every cube value and SED bin within 1e-9 relative, with an
absolute floor of 1e-12 of the largest value (bins deep in the Wien tail).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1112_1071_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    from paper_1112_1071_amd import mcrt

    mcrt.lib()
    return mcrt


def _close(g, o, what):
    floor = 1e-12 * np.max(np.abs(o))
    bad = np.abs(g - o) > 1e-9 * np.abs(o) + floor
    assert not bad.any(), f"{what}: {bad.sum()} of {bad.size} values differ, max rel " \
                          f"{np.max(np.abs(g - o) / (np.abs(o) + floor)):.2e}"


def _compare(M, cfg, T, npix, hw):
    o = oracle.OracleModel(cfg)
    g = M.Model(cfg, precision=M.MCRT_FP64)
    if T is None:  # the GPU's own temperatures after two iterations
        g.iterate()
        g.iterate()
        T = g.temperature()
    else:
        g.set_temperature(T)
    o.set_temperature(T)
    so, co = o.raytrace(npix, hw)
    print(f"raytrace npix {npix} ({len(cfg['peeloff']['dirs'])} observers, {len(cfg['nu_edges']) - 1} bins)",
          flush=True)
    sg, cg = g.raytrace(npix, hw)
    assert cg.shape == co.shape and sg.shape == so.shape
    assert np.any(co > 0) and np.any(so[:, 1] > 0) and np.any(so[:, 0] > 0)
    for i in range(co.shape[0]):
        _close(cg[i], co[i], f"cube, observer {i}")
        _close(sg[i, 0], so[i, 0], f"source SED, observer {i}")
        _close(sg[i, 1], so[i, 1], f"dust SED, observer {i}")
    o.close()
    g.close()
    return sg, cg


def test_raytrace_clump_random_temperatures(M):
    cfg = synth.config2(n=24, n_packets=1000, n_iter=1, n_bins=40, n_src=6, gen_seed=777,
                        box=0.65 * synth.PC * 24 / 128)
    cfg["peeloff"] = {"dirs": [[0.48, -0.6, 0.64], [0.0, 0.0, 1.0], [-0.36, 0.48, -0.8]]}
    rng = np.random.default_rng(11)
    T = np.exp(rng.uniform(math.log(8.0), math.log(400.0), size=np.asarray(cfg["rho"]).size))
    half = 0.5 * 0.65 * synth.PC * 24 / 128
    _compare(M, cfg, T, 37, 1.1 * math.sqrt(3) * half)


def test_raytrace_ragged_grid_cropped_image(M):
    # a non-cubic grid off the origin with empty cells, an image that crops it
    # (rays that miss, rays through edges), sources inside and outside the image
    cfg = synth.config0(n=8, n_packets=1000, n_iter=1, n_bins=30)
    rng = np.random.default_rng(5)
    cfg["grid"] = {"n": [13, 9, 7], "lo": [-3e13, -1e13, 2e12], "hi": [4e13, 2e13, 3.7e13]}
    cfg["rho"] = rng.uniform(0, 3e-15, size=(7, 9, 13)) * (rng.random((7, 9, 13)) > 0.3)
    cfg["sources"] = [{"pos": [1.1e13, 0.3e13, 1.7e13], "lum": synth.L_SUN, "teff": 8000.0},
                      {"pos": [-2.9e13, -0.9e13, 3.0e12], "lum": 0.5 * synth.L_SUN, "teff": 3000.0}]
    cfg["peeloff"] = {"dirs": [[0.6, 0.0, 0.8], [0.0, -1.0, 0.0], [0.48, 0.64, -0.6]]}
    T = rng.uniform(20.0, 300.0, size=13 * 9 * 7)
    _compare(M, cfg, T, 29, 2.2e13)


def test_raytrace_after_iterations(M):
    cfg = synth.config0(n=16, tau=3.0, n_packets=200000, n_iter=2, n_bins=50)
    cfg["peeloff"] = {"dirs": [[0.48, -0.6, 0.64], [0.6, 0.8, 0.0]]}
    _compare(M, cfg, None, 48, 1.05 * math.sqrt(3) * synth.AU)


def test_raytrace_errors(M):
    cfg = synth.config0(n=4, n_packets=100, n_bins=10)
    g = M.Model(cfg)
    with pytest.raises(M.MCRTError):
        g.raytrace(8, synth.AU)  # no observers
    cfg["peeloff"] = {"dirs": [[0.0, 0.0, 1.0]]}
    g = M.Model(cfg)
    with pytest.raises(M.MCRTError):
        g.raytrace(0, synth.AU)
    with pytest.raises(M.MCRTError):
        g.raytrace(8, -1.0)
    sed = np.zeros(2 * 10)
    assert g.L.mcrt_get_raytraced_sed(g.h, sed.ctypes.data, sed.size) == -2  # nothing raytraced yet
    s, _ = g.raytrace(8, synth.AU, cube=False)
    assert s.shape == (1, 2, 10)
    assert g.L.mcrt_get_raytraced_sed(g.h, sed.ctypes.data, sed.size - 1) == -6
