"""Pins of the oracle's grid walk: the summed segment lengths equal the
closed-form chord to the box exit, and the visited cells and lengths equal a
brute-force slab intersection of the ray with every cell on tiny grids."""
import math

import numpy as np
import pytest

import oracle


def tiny_model(n, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0)):
    nu = np.array([1e13, 1e14])
    cfg = {
        "grid": {"n": list(n), "lo": list(lo), "hi": list(hi)},
        "rho": np.ones(int(np.prod(n))),
        "nu_edges": nu,
        "dust": {"chi": np.array([1.0]), "albedo": np.array([0.0]), "g": np.array([0.0])},
        "sources": [{"pos": [0.5 * (lo[a] + hi[a]) for a in range(3)], "lum": 1.0,
                     "spectrum": np.array([1.0])}],
        "observers": {"n_incl": 10},
        "run": {"n_packets": 10},
    }
    return oracle.OracleModel(cfg)


def exit_distance(x, d, lo, hi):
    t = math.inf
    for a in range(3):
        if d[a] > 0:
            t = min(t, (hi[a] - x[a]) / d[a])
        elif d[a] < 0:
            t = min(t, (lo[a] - x[a]) / d[a])
    return t


def brute_force(x, d, n, lo, hi):
    """cells whose box the ray crosses with positive length, by slab tests"""
    dx = [(hi[a] - lo[a]) / n[a] for a in range(3)]
    out = []
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                c = (i, j, k)
                t0, t1 = 0.0, math.inf
                for a in range(3):
                    blo = lo[a] + c[a] * dx[a]
                    bhi = blo + dx[a]
                    if d[a] == 0:
                        if not (blo <= x[a] <= bhi):
                            t0, t1 = 1.0, 0.0
                        continue
                    ta, tb = (blo - x[a]) / d[a], (bhi - x[a]) / d[a]
                    t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
                if t1 - t0 > 1e-9:
                    out.append((t0, i + n[0] * (j + n[1] * k), t1 - t0))
    out.sort()
    return [o[1] for o in out], np.array([o[2] for o in out])


@pytest.mark.parametrize("n", [(1, 1, 1), (2, 2, 2), (3, 2, 4), (4, 4, 4)])
def test_walk_matches_brute_force(n):
    m = tiny_model(n)
    lo, hi = [-1.0] * 3, [1.0] * 3
    rng = np.random.default_rng(sum(n))
    for _ in range(60):
        x = rng.uniform(-0.99, 0.99, 3)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        cells, lens = m.trace_ray(x, d)
        keep = lens > 1e-12
        bc, bl = brute_force(x, d, n, lo, hi)
        assert list(cells[keep]) == bc
        assert np.allclose(lens[keep], bl, rtol=1e-9, atol=1e-12)
        assert lens.sum() == pytest.approx(exit_distance(x, d, lo, hi), rel=1e-12)


def test_chord_length_large_grid():
    n = (17, 9, 31)
    lo, hi = (-3.0, -1.0, 0.5), (2.0, 4.0, 2.0)
    m = tiny_model(n, lo, hi)
    rng = np.random.default_rng(11)
    for _ in range(300):
        x = np.array([rng.uniform(lo[a], hi[a]) for a in range(3)])
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        cells, lens = m.trace_ray(x, d)
        assert np.all(lens >= 0)
        assert lens.sum() == pytest.approx(exit_distance(x, d, lo, hi), rel=1e-12)
        # consecutive cells are face neighbours
        ijk = np.stack(np.unravel_index(cells, n[::-1])[::-1], axis=1)
        steps = np.abs(np.diff(ijk, axis=0)).sum(axis=1)
        assert np.all(steps == 1)


def test_axis_parallel_and_corner_rays():
    n = (4, 4, 4)
    m = tiny_model(n)
    # from the centre (an 8-cell corner) along +x: cells (2..3, 2, 2) of length 0.5
    cells, lens = m.trace_ray(np.zeros(3), np.array([1.0, 0.0, 0.0]))
    assert list(cells) == [2 + 4 * (2 + 4 * 2), 3 + 4 * (2 + 4 * 2)]
    assert np.allclose(lens, 0.5)
    # along -x from the corner: the start cell steps down on x only
    cells, lens = m.trace_ray(np.zeros(3), np.array([-1.0, 0.0, 0.0]))
    assert list(cells) == [1 + 4 * (2 + 4 * 2), 0 + 4 * (2 + 4 * 2)]
    # along the main diagonal from the corner: 2 full cells plus zero-length tie steps
    d = np.array([-1.0, -1.0, -1.0]) / math.sqrt(3)
    cells, lens = m.trace_ray(np.zeros(3), d)
    assert lens.sum() == pytest.approx(math.sqrt(3), rel=1e-12)
    pos = cells[lens > 1e-12]
    assert list(pos) == [1 + 4 * (1 + 4 * 1), 0]
