"""Pins of the warm-start network's CPU reference (oracle/nn.py).

Each convolution geometry is checked against a brute-force sum written from
its definition, the gradients against central finite differences, Adam
against its closed form for a constant gradient, and the features against
values worked out by hand.
"""
import itertools
import math

import numpy as np
import pytest
import torch

from oracle import nn

rng = np.random.default_rng(11)


def _rand(*shape):
    return torch.as_tensor(rng.standard_normal(shape))


def test_conv3_matches_brute_force():
    N, ci, co, D = 2, 3, 2, 4
    x, W, b = _rand(N, ci, D, D, D), _rand(27, co, ci), _rand(co)
    got = nn.conv(nn.CONV3, x, W, b).numpy()
    want = np.zeros((N, co, D, D, D))
    for n, o, z, y, xx in itertools.product(range(N), range(co), range(D), range(D), range(D)):
        s = float(b[o])
        for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
            sz, sy, sx = z + dz, y + dy, xx + dx
            if 0 <= sz < D and 0 <= sy < D and 0 <= sx < D:
                t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                s += float(W[t, o, :] @ x[n, :, sz, sy, sx])
        want[n, o, z, y, xx] = s
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_down_matches_brute_force():
    N, ci, co, D = 1, 2, 3, 4
    x, W, b = _rand(N, ci, D, D, D), _rand(8, co, ci), _rand(co)
    got = nn.conv(nn.DOWN, x, W, b).numpy()
    want = np.zeros((N, co, D // 2, D // 2, D // 2))
    for o, z, y, xx in itertools.product(range(co), range(D // 2), range(D // 2), range(D // 2)):
        s = float(b[o])
        for tz, ty, tx in itertools.product((0, 1), repeat=3):
            s += float(W[tz * 4 + ty * 2 + tx, o, :] @ x[0, :, 2 * z + tz, 2 * y + ty, 2 * xx + tx])
        want[0, o, z, y, xx] = s
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_up_matches_brute_force():
    N, ci, co, D = 1, 3, 2, 2
    x, W, b = _rand(N, ci, D, D, D), _rand(8, co, ci), _rand(co)
    got = nn.conv(nn.UP, x, W, b).numpy()
    want = np.zeros((N, co, 2 * D, 2 * D, 2 * D))
    for o, z, y, xx in itertools.product(range(co), range(D), range(D), range(D)):
        for pz, py, px in itertools.product((0, 1), repeat=3):
            want[0, o, 2 * z + pz, 2 * y + py, 2 * xx + px] = float(b[o]) + float(
                W[pz * 4 + py * 2 + px, o, :] @ x[0, :, z, y, xx])
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def _params(C=16, seed=3):
    r = np.random.default_rng(seed)
    p = []
    for mode, _, _, c1, c2, co, _ in nn.layers(C):
        taps = 27 if mode == nn.CONV3 else 8
        p.append(r.standard_normal(taps * co * (c1 + c2)) * math.sqrt(2.0 / (taps * (c1 + c2))))
        p.append(0.1 * r.standard_normal(co))
    p.append(r.standard_normal(C) / math.sqrt(C))
    p.append([1.5])
    return np.concatenate(p)


def _features(N, D, seed=4):
    r = np.random.default_rng(seed)
    x = np.empty((N * D ** 3, 3), dtype=np.float32)
    x[:, 0] = r.uniform(-6, 2, N * D ** 3)
    x[:, 1] = np.where(r.random(N * D ** 3) < 0.05, r.uniform(1, 9, N * D ** 3), -30.0)
    x[:, 2] = r.uniform(0, 10, N * D ** 3)
    return x


def test_param_count():
    # 3x3x3 levels 16/32/64/128 with skips, 2x2x2 down/up, 1x1x1 head
    assert nn.param_count(16) == 1783585
    p = _params()
    assert p.size == nn.param_count(16)


def test_gradient_matches_finite_differences():
    N, D = 1, 8
    p = _params()
    x = _features(N, D)
    r = np.random.default_rng(5)
    target = r.uniform(1.0, 2.5, N * D ** 3)
    mask = (r.random(N * D ** 3) < 0.7).astype(np.float64)
    loss, g = nn.loss_and_grad(p, x, target, mask, N, D, bf16=False)
    assert np.isfinite(loss) and loss > 0

    def f(q):
        y = nn.forward(q, x, N, D, bf16=False).detach().numpy()
        return float(((y - target) ** 2 * mask).sum() / mask.sum())

    # one weight and one bias of every layer, and the head
    idx = []
    off = 0
    for mode, _, _, c1, c2, co, _ in nn.layers(16):
        nw = (27 if mode == nn.CONV3 else 8) * co * (c1 + c2)
        idx += [off + int(r.integers(nw)), off + nw + int(r.integers(co))]
        off += nw + co
    idx += [off + 3, off + 16]
    for i in idx:
        h = 1e-5 * max(1.0, abs(p[i]))
        qp, qm = p.copy(), p.copy()
        qp[i] += h
        qm[i] -= h
        fd = (f(qp) - f(qm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_bf16_rounding_is_small_and_straight_through():
    N, D = 1, 8
    p = _params()
    x = _features(N, D)
    y0 = nn.forward(p, x, N, D, bf16=False).numpy()
    y1 = nn.forward(p, x, N, D, bf16=True).detach().numpy()
    assert np.abs(y1 - y0).max() < 0.05 and np.abs(y1 - y0).max() > 0


def test_adam_constant_gradient_closed_form():
    # bias correction makes every step lr * g / (|g| + eps) for a constant g
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = v = np.zeros(3)
    q = p.copy()
    for step in range(1, 4):
        q, m, v = nn.adam(q, g, m, v, step, lr=0.01)
    np.testing.assert_allclose(q, p - 3 * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9)


def test_features_by_hand():
    n = 8
    half = 4.0
    rho = np.zeros((n, n, n))
    rho[2, 3, 1] = 0.5  # k, j, i
    cfg = {
        "grid": {"n": [n] * 3, "lo": [-half] * 3, "hi": [half] * 3},
        "rho": rho,
        "nu_edges": np.array([1e12, 2e14, 1e15, 1e16]),  # 1 um = 3e14 Hz lies in bin 1
        "dust": {"chi": np.array([1.0, 2.0, 3.0])},
        "sources": [{"pos": [0.0, 0.0, 0.0], "lum": 8.0},        # a corner of 8 cells
                    {"pos": [0.5, -2.5, 1.25], "lum": 4.0 * math.pi}],  # inside cell (4, 1, 5)
    }
    x = nn.features(cfg)
    dx = 1.0
    tau = x[:, 0].reshape(n, n, n)
    assert tau[2, 3, 1] == pytest.approx(math.log10(0.5 * 2.0 * dx))
    assert tau[0, 0, 0] == pytest.approx(-6.0)
    F = 10 ** x[:, 1].reshape(n, n, n)
    for k, j, i in itertools.product((3, 4), repeat=3):
        assert F[k, j, i] == pytest.approx(1.0 / (4 * math.pi))
    assert F[5, 1, 4] == pytest.approx(1.0)
    assert (F > 1e-20).sum() == 9
    # spread field: sum of D_c / max(r^2, 1/4) over the 9 deposit cells
    G = 10 ** x[:, 2].reshape(n, n, n)
    dep = [((i, j, k), 1.0 / (4 * math.pi)) for k, j, i in itertools.product((3, 4), repeat=3)]
    dep.append(((4, 1, 5), 1.0))
    for (k, j, i) in [(0, 0, 0), (5, 1, 4), (3, 3, 3), (7, 2, 6)]:
        want = sum(d / max((i - a) ** 2 + (j - b) ** 2 + (k - c) ** 2, 0.25) for (a, b, c), d in dep)
        assert G[k, j, i] == pytest.approx(want, rel=1e-12)
