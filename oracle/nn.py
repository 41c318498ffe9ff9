"""FP64 CPU reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

The tests and ``__graft_entry__.smoke()`` may use it; the product path never
does.  It imports nothing from the HIP package.

What it computes (the network that warm-starts the Lucy temperature iteration
of Sec. 2.4): a 3-D convolutional encoder-decoder on N cubes of side D,

* input: three features per cell, shifted and scaled, channel 0 -> (x0 + 2) / 2,
  channel 1 -> (x1 + 30) / 10, channel 2 -> (x2 - 4) / 3, zero-padded to 16
  channels;
* level l (l = 0..3) has C * 2^l channels; encoder levels 0-2: two 3x3x3
  convolutions (zero padding 1) then a 2x2x2 stride-2 convolution; level 3:
  two 3x3x3 convolutions; decoder levels 2..0: a 2x2x2 stride-2 transposed
  convolution, concatenation [upsampled, skip] along channels, two 3x3x3
  convolutions; every convolution adds a bias and applies LeakyReLU(0.1);
* a 1x1x1 head to one channel: log10 T.

Parameters are one flat FP32 vector, per layer in the order above: weights
[taps][C_out][C_in] (3x3x3 tap = dz*9 + dy*3 + dx over offsets -1..1; 2x2x2
tap = tz*4 + ty*2 + tx) then biases [C_out]; the head's weights [C] and bias.

The matrix-core path rounds weights, inputs and every activation to BF16
(round to nearest even) and accumulates in FP32; ``forward(..., bf16=True)``
applies the same roundings in FP64 arithmetic, with straight-through gradients
(the rounding is the identity for backpropagation).  Convolutions are the
library routines ``torch.nn.functional.conv3d`` / ``conv_transpose3d`` in FP64
on the CPU; the tests pin their use against brute-force sums written from the
definitions above, and the gradients against central finite differences.
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

SLOPE = 0.1
NORM = (2.0, 0.5, 30.0, 0.1, -4.0, 1.0 / 3.0)
CONV3, DOWN, UP = 0, 1, 2


def layers(C: int = 16):
    """[(mode, in1, in2, C_in1, C_in2, C_out, out_tensor)], tensor channels."""
    tens = [16]  # tensor 0: padded input
    out = []

    def add(mode, a, b, cout):
        tens.append(cout)
        out.append((mode, a, b, tens[a], tens[b] if b >= 0 else 0, cout, len(tens) - 1))
        return len(tens) - 1

    t = add(CONV3, 0, -1, C)
    s0 = add(CONV3, t, -1, C)
    t = add(DOWN, s0, -1, 2 * C)
    t = add(CONV3, t, -1, 2 * C)
    s1 = add(CONV3, t, -1, 2 * C)
    t = add(DOWN, s1, -1, 4 * C)
    t = add(CONV3, t, -1, 4 * C)
    s2 = add(CONV3, t, -1, 4 * C)
    t = add(DOWN, s2, -1, 8 * C)
    t = add(CONV3, t, -1, 8 * C)
    t = add(CONV3, t, -1, 8 * C)
    t = add(UP, t, -1, 4 * C)
    t = add(CONV3, t, s2, 4 * C)
    t = add(CONV3, t, -1, 4 * C)
    t = add(UP, t, -1, 2 * C)
    t = add(CONV3, t, s1, 2 * C)
    t = add(CONV3, t, -1, 2 * C)
    t = add(UP, t, -1, C)
    t = add(CONV3, t, s0, C)
    t = add(CONV3, t, -1, C)
    return out


def param_count(C: int = 16) -> int:
    n = 0
    for mode, _, _, c1, c2, co, _ in layers(C):
        n += (27 if mode == CONV3 else 8) * co * (c1 + c2) + co
    return n + C + 1


def unpack(p, C: int = 16):
    """flat vector -> [(W [taps][C_out][C_in], b)], head_w, head_b (torch FP64)."""
    p = torch.as_tensor(np.asarray(p, dtype=np.float64))
    off = 0
    out = []
    for mode, _, _, c1, c2, co, _ in layers(C):
        taps = 27 if mode == CONV3 else 8
        nw = taps * co * (c1 + c2)
        W = p[off:off + nw].reshape(taps, co, c1 + c2)
        off += nw
        b = p[off:off + co]
        off += co
        out.append((W, b))
    hw = p[off:off + C]
    hb = p[off + C]
    assert off + C + 1 == p.numel()
    return out, hw, hb


def _bf16(x, on: bool):
    if not on:
        return x
    r = x.to(torch.bfloat16).to(torch.float64)
    return x + (r - x).detach()


class _RoundGrad(torch.autograd.Function):
    """Identity forward; backward rounds the incoming gradient to BF16 (the
    matrix-core training path stores each layer's pre-activation gradient
    in BF16)."""

    @staticmethod
    def forward(ctx, x):
        return x.view_as(x)

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.bfloat16).to(torch.float64)


def conv(mode: int, x, W, b, fp32: bool = False):
    """One convolution in NCDHW FP64; W [taps][C_out][C_in] as in the layout.
    fp32: accumulate in FP32 instead (the result is returned as FP64)."""
    if fp32:
        return conv(mode, x.float(), W.float(), b.float()).double()
    co, ci = W.shape[1], W.shape[2]
    if mode == CONV3:
        w = W.reshape(3, 3, 3, co, ci).permute(3, 4, 0, 1, 2)
        return F.conv3d(x, w, b, padding=1)
    if mode == DOWN:
        w = W.reshape(2, 2, 2, co, ci).permute(3, 4, 0, 1, 2)
        return F.conv3d(x, w, b, stride=2)
    w = W.reshape(2, 2, 2, co, ci).permute(4, 3, 0, 1, 2)  # [C_in][C_out][kz][ky][kx]
    return F.conv_transpose3d(x, w, b, stride=2)


def inputs(x, N: int, D: int, bf16: bool = True):
    """features [N*D^3, 3] (FP32 values) -> padded NCDHW input tensor."""
    x = torch.as_tensor(np.asarray(x, dtype=np.float32).astype(np.float64)).reshape(N, D, D, D, 3)
    t = torch.zeros((N, 16, D, D, D), dtype=torch.float64)
    for c in range(3):
        t[:, c] = _bf16((x[..., c] + NORM[2 * c]) * NORM[2 * c + 1], bf16)
    return t


def forward(p, x, N: int, D: int, C: int = 16, bf16: bool = True, params_grad: bool = False,
            bf16_grad: bool = False, fp32: bool = False):
    """log10 T [N*D^3] (and the torch parameter leaves when params_grad).
    bf16_grad: round each layer's pre-activation gradient to BF16 in the
    backward pass, as the matrix-core training path does.  fp32: accumulate
    the convolutions in FP32 (another admissible order of the same roundings;
    the spread between the two measures how sensitive a result is to it)."""
    lw, hw, hb = unpack(p, C)
    leaves = []
    if params_grad:
        lw = [(W.clone().requires_grad_(True), b.clone().requires_grad_(True)) for W, b in lw]
        hw = hw.clone().requires_grad_(True)
        hb = hb.clone().requires_grad_(True)
        leaves = [t for wb in lw for t in wb] + [hw, hb]
    T = [inputs(x, N, D, bf16)]
    for (mode, a, b2, _, _, _, _), (W, b) in zip(layers(C), lw):
        inp = T[a] if b2 < 0 else torch.cat([T[a], T[b2]], dim=1)
        z = conv(mode, inp, _bf16(W, bf16), b, fp32)
        if bf16_grad:
            z = _RoundGrad.apply(z)
        T.append(_bf16(F.leaky_relu(z, SLOPE), bf16))
    y = torch.einsum("ncdhw,c->ndhw", T[-1], hw) + hb
    y = y.reshape(-1)
    return (y, leaves) if params_grad else y


def loss_and_grad(p, x, target, mask, N: int, D: int, C: int = 16, bf16: bool = True,
                  bf16_grad: bool = False, fp32: bool = False):
    """sum mask (y - t)^2 / sum mask and its gradient as a flat FP64 vector."""
    y, leaves = forward(p, x, N, D, C, bf16, params_grad=True, bf16_grad=bf16_grad, fp32=fp32)
    t = torch.as_tensor(np.asarray(target, dtype=np.float64))
    m = torch.as_tensor(np.asarray(mask, dtype=np.float64))
    loss = ((y - t) ** 2 * m).sum() / m.sum()
    loss.backward()
    g = torch.cat([lf.grad.reshape(-1) for lf in leaves])
    return float(loss.detach()), g.numpy()


def adam(p, g, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected moments), FP64; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(cfg: dict) -> np.ndarray:
    """Network features of a model config, FP64 [ncell, 3]: log10 of the cell
    optical depth at 1 micron (floored at 1e-6); log10(D + 1e-30), D the
    deposit field (luminosity of the sources in the cell over 4 pi dx^2; a
    source on a cell wall, edge or corner is shared equally by the cells
    touching it); log10 of the deposit field spread by the free-space kernel,
    sum over deposit cells of D_c dx^2 / max(r^2, dx^2/4) with r the distance
    between cell centres, + 1e-30."""
    n = [int(v) for v in cfg["grid"]["n"]]
    lo = np.asarray(cfg["grid"]["lo"], dtype=np.float64)
    hi = np.asarray(cfg["grid"]["hi"], dtype=np.float64)
    dx = (hi - lo) / np.asarray(n)
    nu = np.asarray(cfg["nu_edges"], dtype=np.float64)
    nu1 = 2.99792458e10 / 1e-4
    k = int(np.searchsorted(nu, nu1, side="right") - 1)
    k = min(max(k, 0), len(nu) - 2)
    chi1 = float(np.asarray(cfg["dust"]["chi"])[k])
    rho = np.asarray(cfg["rho"], dtype=np.float64).reshape(-1)
    tau = np.maximum(rho * chi1 * dx[0], 1e-6)
    lum = np.zeros(rho.size)
    for s in cfg["sources"]:
        ranges = []
        for a in range(3):
            f = (s["pos"][a] - lo[a]) / dx[a]
            c = int(math.floor(f))
            cells = [min(max(c, 0), n[a] - 1)]
            if f == math.floor(f) and 0 < c < n[a]:
                cells = [c - 1, c]
            ranges.append(cells)
        cnt = len(ranges[0]) * len(ranges[1]) * len(ranges[2])
        for kk in ranges[2]:
            for j in ranges[1]:
                for i in ranges[0]:
                    lum[i + n[0] * (j + n[1] * kk)] += s["lum"] / cnt
    dep = lum / (4.0 * math.pi * dx[0] ** 2)
    kk, jj, ii = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    ii, jj, kk = ii.reshape(-1), jj.reshape(-1), kk.reshape(-1)
    spread = np.zeros(rho.size)
    for c in np.nonzero(dep)[0]:
        r2 = (ii - ii[c]) ** 2 + (jj - jj[c]) ** 2 + (kk - kk[c]) ** 2
        spread += dep[c] / np.maximum(r2, 0.25)
    return np.stack([np.log10(tau), np.log10(dep + 1e-30), np.log10(spread + 1e-30)], axis=1)
