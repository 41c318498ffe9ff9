"""Warm-start network on the matrix cores against the FP64 CPU reference.

Forward outputs, the loss, every parameter gradient and one Adam step of the
library's BF16/FP32 kernels are compared with oracle/nn.py evaluated with
the same BF16 roundings of weights, inputs and activations.

Tolerances (from the arithmetic): both sides round weights, inputs,
activations and each layer's pre-activation gradient to BF16 at the same
points, so they differ only where FP32 (GPU) and FP64 (reference)
accumulation put a value on different sides of a BF16 rounding boundary.
Such a flip changes one element by one BF16 unit (2^-8 relative), and flips
propagate: through the forward pass to log10 T (bar 1e-2 absolute, median
1e-3), and through activation-derivative masks into the gradients of the
deep layers, whose small gradients can move by 10 % between two admissible
rounding orders.  The bar per parameter tensor is therefore a relative L2
error below max(2e-2, 3 s), where s is the reference's own spread for that
tensor between FP64 and FP32 accumulation; a wrong index, tap or operand
gives errors of order 1.
"""
import numpy as np
import pytest

from oracle import nn
from paper_1112_1071_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    from paper_1112_1071_amd import mcrt

    mcrt.lib()
    return mcrt


def _features(N, D, seed):
    r = np.random.default_rng(seed)
    x = np.empty((N * D ** 3, 3), dtype=np.float32)
    x[:, 0] = r.uniform(-6, 2, N * D ** 3)
    x[:, 1] = np.where(r.random(N * D ** 3) < 0.05, r.uniform(1, 9, N * D ** 3), -30.0)
    x[:, 2] = r.uniform(0, 10, N * D ** 3)
    return x


def _layer_slices(C=16):
    out = []
    off = 0
    for i, (mode, _, _, c1, c2, co, _) in enumerate(nn.layers(C)):
        nw = (27 if mode == nn.CONV3 else 8) * co * (c1 + c2)
        out.append((f"L{i}.w", slice(off, off + nw)))
        out.append((f"L{i}.b", slice(off + nw, off + nw + co)))
        off += nw + co
    out.append(("head.w", slice(off, off + C)))
    out.append(("head.b", slice(off + C, off + C + 1)))
    return out


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


# N x D: several MFMA row tiles with ragged tails at every level (D = 24:
# 3^3 = 27 voxels at the coarsest level), and the 1-voxel bottleneck (D = 8)
@pytest.mark.parametrize("N,D", [(1, 8), (2, 16), (1, 24)])
def test_forward_and_gradients_match_reference(M, N, D):
    import torch

    sur = M.Surrogate(0, 16, seed=7 + D)
    p = sur.params().astype(np.float64)
    assert p.size == nn.param_count(16)
    x = _features(N, D, seed=D)
    r = np.random.default_rng(100 + D)
    target = r.uniform(1.0, 2.5, N * D ** 3).astype(np.float32)
    mask = (r.random(N * D ** 3) < 0.7).astype(np.float32)
    dev = "cuda:0"
    xt = torch.as_tensor(x, device=dev).contiguous()
    tt = torch.as_tensor(target, device=dev)
    mt = torch.as_tensor(mask, device=dev)

    y = sur.forward(xt, N, D).cpu().numpy()
    y_ref = nn.forward(p, x, N, D).detach().numpy()
    assert np.abs(y - y_ref).max() < 1e-2
    assert np.median(np.abs(y - y_ref)) < 1e-3

    loss = sur.train_step(xt, tt, mt, N, D, lr=0.0, apply_update=False)
    loss_ref, g_ref = nn.loss_and_grad(p, x, target, mask, N, D, bf16_grad=True)
    _, g_ref32 = nn.loss_and_grad(p, x, target, mask, N, D, bf16_grad=True, fp32=True)
    assert loss == pytest.approx(loss_ref, rel=2e-2)
    g = sur.grads().astype(np.float64)
    # input channels 3..15 are zero: their first-layer weights get zero gradient
    assert not np.any(g[_layer_slices()[0][1]].reshape(27, 16, 16)[:, :, 3:])
    rows = []
    for name, sl in _layer_slices():
        e, spread = _rel(g[sl], g_ref[sl]), _rel(g_ref32[sl], g_ref[sl])
        rows.append((name, round(e, 5), round(spread, 5)))
        assert e < max(2e-2, 3 * spread), (name, e, spread)
    print("gradient error / reference spread per tensor:", rows)

    # one Adam step, against the closed-form update from the gradients that
    # step computed: the weight gradients are FP32 atomic sums, so a second
    # evaluation differs in its last bits, and the first Adam step,
    # lr g / (|g| + eps), magnifies that for gradients near eps
    lr = 1e-3
    sur.train_step(xt, tt, mt, N, D, lr=lr, apply_update=True)
    g = sur.grads().astype(np.float64)
    q_ref, _, _ = nn.adam(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr)
    q = sur.params().astype(np.float64)
    np.testing.assert_allclose(q, q_ref, rtol=1e-5, atol=1e-7)
    # the forward pass sees the new BF16 weights
    y2 = sur.forward(xt, N, D).cpu().numpy()
    y2_ref = nn.forward(q, x, N, D).detach().numpy()
    assert np.abs(y2 - y2_ref).max() < 1e-2
    sur.close()


def test_gradient_clipping(M):
    import torch

    N, D = 1, 8
    sur = M.Surrogate(0, 16, seed=5)
    p = sur.params().astype(np.float64)
    x = torch.as_tensor(_features(N, D, seed=3), device="cuda:0").contiguous()
    r = np.random.default_rng(9)
    t = torch.as_tensor(r.uniform(1, 2.5, D ** 3).astype(np.float32), device="cuda:0")
    k = torch.ones(D ** 3, dtype=torch.float32, device="cuda:0")
    sur.train_step(x, t, k, N, D, lr=0.0, apply_update=False)
    g = sur.grads().astype(np.float64)
    clip = 0.25 * np.linalg.norm(g)
    sur.set_grad_clip(clip)
    sur.train_step(x, t, k, N, D, lr=1e-3, apply_update=True)
    g = sur.grads().astype(np.float64)  # the gradients of this step (FP32 atomic sums)
    assert np.linalg.norm(g) > clip
    q_ref, _, _ = nn.adam(p, g * clip / np.linalg.norm(g), np.zeros_like(p), np.zeros_like(p), 1, 1e-3)
    np.testing.assert_allclose(sur.params().astype(np.float64), q_ref, rtol=1e-5, atol=1e-7)
    with pytest.raises(M.MCRTError):
        sur.set_grad_clip(-1.0)
    sur.close()


def test_set_params_roundtrip_and_errors(M):
    sur = M.Surrogate(0, 16, seed=1)
    p = sur.params()
    q = (p * 0.5).astype(np.float32)
    sur.set_params(q)
    assert np.array_equal(sur.params(), q)
    with pytest.raises(M.MCRTError):
        sur.set_params(q[:-1])
    bad = q.copy()
    bad[5] = np.nan
    with pytest.raises(M.MCRTError):
        sur.set_params(bad)
    import torch

    x = torch.zeros((12 ** 3, 3), device="cuda:0")
    with pytest.raises(M.MCRTError):
        sur.forward(x, 1, 12)  # side not a multiple of 8
    sur.close()


def test_model_features_match_reference(M):
    cfg = synth.config2(n=32, n_packets=1000, n_iter=1, gen_seed=45123, n_src=20, box=0.65 * synth.PC / 4)
    # a source on a cell corner and one on a wall
    lo, hi = cfg["grid"]["lo"][0], cfg["grid"]["hi"][0]
    dx = (hi - lo) / 32
    cfg["sources"][0]["pos"] = [lo + 10 * dx, lo + 12 * dx, lo + 7 * dx]
    cfg["sources"][1]["pos"] = [lo + 3.5 * dx, lo + 20 * dx, lo + 30.5 * dx]
    m = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT)
    x = m.features().cpu().numpy()
    ref = nn.features(cfg)
    np.testing.assert_allclose(x[:, 0], ref[:, 0], rtol=0, atol=2e-6)
    np.testing.assert_allclose(x[:, 1], ref[:, 1], rtol=0, atol=1e-5)
    np.testing.assert_allclose(x[:, 2], ref[:, 2], rtol=0, atol=1e-5)
    assert np.count_nonzero(ref[:, 1] > -29) == np.count_nonzero(x[:, 1] > -29)


def test_warm_start_sets_network_temperatures(M):
    cfg = synth.clump_config4(n=32, seed=45999, n_src=10, n_packets=200000, n_iter=2)
    m = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT)
    sur = M.Surrogate(0, 16, seed=3)
    ms = m.warm_start(sur)
    assert ms > 0
    y = sur.forward(m.features(), 1, 32).cpu().numpy()
    T0 = np.clip(10.0 ** y.astype(np.float64), 1.0, 1e4)
    # the first iteration re-emits from the network's temperatures
    np.testing.assert_allclose(m.temperature(), T0, rtol=1e-12)
    st = m.iterate()
    assert st["iteration"] == 0
    bad = synth.config0(n=12, n_packets=1000)
    mb = M.Model(bad, precision=M.MCRT_FP32_TRANSPORT)
    with pytest.raises(M.MCRTError):
        mb.warm_start(sur)
    sur.close()
