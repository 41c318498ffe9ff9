"""Error bound of the raytracing's Planck table (Sec. 2.6.3 source function).

The GPU raytracer reads B_k(T), the Planck function integrated over bin k,
from a table of ln B_k on 2048 rows uniform in ln T over 1..1e4 K, holding
values and slopes d ln B_k / d ln T = (4 I + a f(a) - b f(b)) / I (I the bin
integral of f(x) = x^3 / (e^x - 1) over [a, b], x = h nu / k T), and
interpolates cubic Hermite in ln T.  The remainder of cubic Hermite is
h^4 / 384 max |g''''|, h = ln(1e4) / 2047, with g = ln B_k; on the Wien side
g is about -x plus slowly varying terms, so |g''''| is about x, and the
relative error is about 1.1e-12 max(x, 1).  Checked here against the
oracle's own bin integral (its series) at random temperatures over the
200-bin grid of the disk and clump models: the bar is 3e-12 max(x, 1).
"""
import ctypes as C

import numpy as np

import oracle
from paper_1112_1071_amd import synth

H, K, CL = 6.62607015e-27, 1.380649e-16, 2.99792458e10
ROWS = 2048
DL = np.log(1e4) / (ROWS - 1)


def _lib():
    L = oracle.lib()
    L.orc_planck_x_integral.restype = C.c_double
    L.orc_planck_x_integral.argtypes = [C.c_double, C.c_double]
    return L


def _f(x):
    if not 0.0 < x < 745.0:
        return 0.0
    return x ** 3 * np.exp(-x) if x > 700.0 else x ** 3 / np.expm1(x)


def _ln_b(L, nu, T):
    """ln B_k, d ln B_k / d ln T and x_lo per bin (nan where B underflows)"""
    kT = K * T
    pref = 2.0 * kT ** 4 / (H ** 3 * CL ** 2)
    out = np.full((len(nu) - 1, 3), np.nan)
    for i in range(len(nu) - 1):
        a, b = H * nu[i] / kT, H * nu[i + 1] / kT
        I = L.orc_planck_x_integral(a, b)
        out[i, 2] = a
        if pref * I > 1e-300:
            out[i, 0] = np.log(pref * I)
            out[i, 1] = (4.0 * I + a * _f(a) - b * _f(b)) / I
    return out


def test_hermite_table_of_ln_b_meets_its_bound():
    L = _lib()
    nu = synth.nu_edges_log(200)
    rng = np.random.default_rng(3)
    worst = 0.0
    for T in np.exp(rng.uniform(0.0, np.log(1e4), 12)):
        u = np.log(T) / DL
        r = min(int(u), ROWS - 2)
        f = u - r
        e0, e1, ex = _ln_b(L, nu, np.exp(r * DL)), _ln_b(L, nu, np.exp((r + 1) * DL)), _ln_b(L, nu, T)
        f2, f3 = f * f, f ** 3
        g = ((2 * f3 - 3 * f2 + 1) * e0[:, 0] + (f3 - 2 * f2 + f) * DL * e0[:, 1] +
             (-2 * f3 + 3 * f2) * e1[:, 0] + (f3 - f2) * DL * e1[:, 1])
        ok = np.isfinite(g) & np.isfinite(ex[:, 0])
        assert ok.sum() > 20
        rel = np.abs(np.expm1(g[ok] - ex[ok, 0])) / np.maximum(ex[ok, 2], 1.0)
        worst = max(worst, rel.max())
    assert worst < 3e-12, worst
