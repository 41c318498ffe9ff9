#!/usr/bin/env python3
"""Benchmark: packets/s of Lucy iterations on the 256^3 star-forming clump.

One step = one Lucy iteration over one batch of packets (emission, grid walk
with the path-length estimator, scatter/absorb/re-emit, escape; then Adot, the
LTE temperature update and the convergence statistics), on one GPU, with all
inputs resident in device memory.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--packets N] [--precision fp32|fp64]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA, published


def algorithmic_bytes(st: dict, precision: int) -> float:
    """Bytes the method must move per launch: per dust-cell segment a density
    gather (4 B FP32 / 8 B FP64) and an FP64 read-modify-write of the cell's
    absorption tally (16 B); per empty-cell segment the density gather; per
    absorption the cell's emission-row position (4 B / 8 B)."""
    rb = 4 if precision == 1 else 8
    return (st["n_cross_dust"] * (rb + 16) + st["n_cross_empty"] * rb + st["n_absorb"] * rb)


def measured_traffic(precision: int, mode: int, workload: str = "clump256"):
    """HBM bytes per pass of the dominant transport kernel (the sweeps and the
    tail's finish, or the per-lane walk), and per pass of every transport
    kernel, from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if it
    was taken on the current transport source, in the same precision and
    transport mode."""
    from paper_1112_1071_amd.profiling import transport_source_hash

    p = os.path.join(ROOT, "profiles", "transport_clump256_pmc.json")
    if not os.path.exists(p):
        return None, None
    try:
        d = json.load(open(p))
    except Exception:
        return None, None
    if (d.get("source_hash") != transport_source_hash() or d.get("precision") != precision
            or d.get("mode") != mode or d.get("workload", "clump256") != workload):
        return None, None
    return d.get("dominant_bytes_per_pass"), d.get("hbm_bytes_per_pass")


def cpu_baseline(cfg: dict, n_packets: int, what: str, one_thread_packets: int = 0) -> dict:
    """The oracle's transport on the host cores: a bounded sample of a first
    Lucy iteration of the same model, on all cores (and, when asked, on one)."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    o = oracle.OracleModel(cfg, n_threads=threads)
    st = o.transport_sample(n_packets)
    o.close()
    out = {"value": n_packets / st["seconds"], "unit": "packets/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{n_packets} packets of a first Lucy iteration of the same {what} "
                     f"(FP64 oracle transport only, {st['seconds']:.1f} s)"}
    if one_thread_packets:
        o = oracle.OracleModel(cfg, n_threads=1)
        s1 = o.transport_sample(one_thread_packets)
        o.close()
        out["one_thread"] = {"value": one_thread_packets / s1["seconds"], "packets": one_thread_packets,
                             "seconds": s1["seconds"]}
    return out


def bench_batch(args):
    """Form 2: the batched family of uneven models, one persistent launch per
    Lucy iteration (graph-replayed, autotuned) vs one launch per model.  Both
    sides run iteration 0 untimed and then time the same iterations 1..steps
    (an iteration's cost grows as the dust warms up)."""
    from paper_1112_1071_amd import mcrt, synth
    import torch

    t0 = time.time()
    cfgs = [synth.config3_model(m, packets_per_cell=args.ppc, n_iter=args.steps + 1)
            for m in range(args.models)]
    print(f"# {args.models} models built in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    prec = mcrt.MCRT_FP32_TRANSPORT if args.precision != "fp64" else mcrt.MCRT_FP64
    extra = {"mrw_gamma": args.mrw} if args.mrw > 0 else {}
    if args.tally_copies:
        extra["tally_copies"] = args.tally_copies
    if args.max_events:
        extra["max_events"] = args.max_events
    batch = [mcrt.Model(c, precision=prec, **extra) for c in cfgs]
    n_packets = sum(int(c["run"]["n_packets"]) for c in cfgs)
    cells = sum(int(np.prod(c["grid"]["n"])) for c in cfgs)
    # launch shape: given in full, or tuned (cached per workload class)
    shape = dict(autotune=1)
    if args.block_size and args.walk_batch and args.defer:
        shape = dict(autotune=0, block_size=args.block_size, walk_batch=args.walk_batch,
                     defer_lanes=args.defer)
    # iteration 0, which also tunes the launch shape
    stw = mcrt.batch_run(batch, n_iter=1, final_pass=0, use_graph=0, verbose=1, **shape)
    print(f"# iteration 0 + tuning: {stw['ms_total']:.0f} ms (tune {stw['ms_tune']:.0f} ms) shape "
          f"bs={stw['block_size']} K={stw['walk_batch']} defer={stw['defer_lanes']}",
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    st = mcrt.batch_run(batch, n_iter=args.steps, final_pass=0, use_graph=1, verbose=1, **shape)
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - tb
    value = n_packets * args.steps / batch_s
    print(f"# batched: {1e3 * batch_s / args.steps:.1f} ms per iteration", file=sys.stderr, flush=True)
    del batch
    # the same iterations, one model at a time: with the batched launch's own
    # walk (per-lane, transport_mode 0), and with the tiled sweeps (the
    # single-model default)
    nseq = min(args.seq_models, args.models)
    seq = {}
    for mode in (0, 1):
        seq_s, seq_packets = 0.0, 0
        for i, c in enumerate(cfgs[:nseq]):
            m = mcrt.Model(c, precision=prec, transport_mode=mode, **extra)
            m.iterate()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for _ in range(args.steps):
                m.iterate()
            torch.cuda.synchronize()
            seq_s += time.perf_counter() - ts
            seq_packets += int(c["run"]["n_packets"]) * args.steps
            m.close()
            if (i + 1) % 8 == 0:
                print(f"# sequential, transport_mode {mode}: {i + 1}/{nseq} models", file=sys.stderr,
                      flush=True)
        seq[mode] = {"value": seq_packets / seq_s if nseq else None, "unit": "packets/s",
                     "models": nseq, "seconds": seq_s, "transport_mode": mode}
    # the batched rate over the same models as the sequential legs, when they
    # cover them all
    for mode in (0, 1):
        seq[mode]["speedup_batched"] = value / seq[mode]["value"] if nseq == args.models else None
    print(f"# sequential: {seq[0]['value']} / {seq[1]['value']} packets/s (per-lane walk / tiled)",
          file=sys.stderr, flush=True)
    ms_it = 1e3 * batch_s / args.steps
    out = {
        "metric": "packets/s, batched Lucy iterations of uneven models",
        "value": value, "unit": "packets/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": ms_it, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32" if prec == 1 else "fp64", "data": "synthetic",
        "config": {"workload": f"batch{args.models}: {args.models} models, grids 16^3..96^3 "
                               f"({cells} cells), sphere/disk family, {args.ppc} packets per cell "
                               f"per iteration ({n_packets:.3e} packets), iterations 1..{args.steps}"
                               + (f", modified random walk gamma {args.mrw}" if args.mrw > 0 else ""),
                   "models": args.models, "packets_per_step": n_packets},
        "batch": {"graph_used": st["graph_used"], "tuned": st["tuned"],
                  "block_size": st["block_size"], "walk_batch": st["walk_batch"],
                  "defer_lanes": st["defer_lanes"], "blocks_per_cu": st["blocks_per_cu"],
                  "ms_tune": stw["ms_tune"]},
        "sequential": seq[1], "sequential_per_lane_walk": seq[0],
    }
    print(json.dumps(out), flush=True)


def bench_raytrace(args):
    """Raytracing (Sec. 2.6.3) of the 256^3 clump's dust and source emission in
    all 200 bins toward one oblique observer, npix^2 rays, at the temperatures
    of two Lucy iterations of 1e7 packets."""
    from paper_1112_1071_amd import mcrt, synth

    cfg = synth.config2(n=args.grid, n_packets=10_000_000, n_iter=2)
    cfg["peeloff"] = {"dirs": [[0.48, -0.6, 0.64]]}
    m = mcrt.Model(cfg, precision=mcrt.MCRT_FP32_TRANSPORT)
    m.iterate()
    m.iterate()
    hw = 0.5 * 0.65 * synth.PC * math.sqrt(3.0) * 1.01
    m.raytrace(args.npix, hw, cube=False)  # warm-up (allocation)
    times = []
    for i in range(args.steps):
        t0 = time.perf_counter()
        sed, _ = m.raytrace(args.npix, hw, cube=False)
        times.append(time.perf_counter() - t0)
        print(f"# raytrace {i}: {1e3 * times[-1]:.1f} ms", file=sys.stderr, flush=True)
    ms = 1e3 * float(np.median(times))
    nnu = len(cfg["nu_edges"]) - 1
    # cell segments of all rays: every ray through the grid box crosses about
    # (chord / cell) * (|o_x| + |o_y| + |o_z|) cells; counted exactly by the oracle's walk
    # would cost minutes, so the figure uses the mean chord of the image's rays
    n = args.grid
    o = np.array([0.48, -0.6, 0.64])
    cells_per_length = np.abs(o).sum() * n / (0.65 * synth.PC)
    mean_chord_area = (0.65 * synth.PC) ** 3  # sum over rays of chord * pixel area = volume
    apix = (2 * hw / args.npix) ** 2
    segments = mean_chord_area / apix * cells_per_length
    out = {
        "metric": "raytraced emission: cell-bin segments per second",
        "value": segments * nnu / (ms * 1e-3), "unit": "segments/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"raytrace: {n}^3 clump, {nnu} bins, one observer, {args.npix}^2 rays",
                   "npix": args.npix, "rays": args.npix ** 2, "cell_segments": segments,
                   "sed_dust_total": float(sed[0, 1].sum()), "sed_sources_total": float(sed[0, 0].sum())},
    }
    print(json.dumps(out), flush=True)


def bench_pda(args):
    """Partial diffusion approximation (Sec. 2.3, Appendix A) on the poorly
    sampled mid-plane of the 128^3 disk at mid-plane tau(1 um) = 1e4 after one
    Lucy iteration of 1e6 packets: selection, conjugate-gradient solves of the
    T^4 system (matrix-free 7-point stencil) and the new temperatures."""
    import torch

    from paper_1112_1071_amd import mcrt, synth

    cfg = synth.config1(n=128, tau=1e4, n_packets=1_000_000, n_iter=1, npix=8)
    m = mcrt.Model(cfg, precision=mcrt.MCRT_FP64, want_noise=1)
    m.iterate()
    T0 = m.temperature()
    stats = []
    for i in range(args.warmup + args.steps):
        m.set_temperature(T0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = m.apply_pda(0.1, passes=3)
        torch.cuda.synchronize()
        if i >= args.warmup:
            stats.append((time.perf_counter() - t0) * 1e3)
    ms = float(np.mean(stats))
    nc = 128 ** 3
    # per CG iteration and cell: flags 8 B, the 7-point stencil's 7 x 8 B of p,
    # 3 x 8 B of vectors read or written
    it = st["cg_iterations"] * st["passes"]
    gbs = it * nc * 88.0 / (ms * 1e-3) / 1e9
    out = {
        "metric": "partial diffusion approximation: solve time", "value": ms, "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "pda: 128^3 disk, mid-plane tau(1 um) = 1e4, after one iteration of 1e6 "
                               "packets; cells with sigma_Adot/Adot > 0.1 or unsampled", "grid": 128},
        "roofline": {"bound": "hbm", "kernel": "k_pda_apply + k_pda_step", "achieved": gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "note": "88 B per cell per CG iteration, over the whole call (selection included)"},
        "pda": st,
    }
    print(json.dumps(out), flush=True)


def surrogate_flops(N: int, D: int, C0: int = 16) -> dict:
    """Multiply-add FLOPs (2 per MAC) of one forward pass and of one training
    step of the warm-start network on N cubes of side D: every convolution is a
    GEMM of rows x taps*Cin x Cout (the first layer's 3 features padded to 16
    channels, as the kernels run it); a step is the forward pass, the
    backward-data pass (all layers but the first) and the weight gradients."""
    # (mode, Cin, Cout, level of the GEMM rows): CONV3 27 taps over output
    # voxels, DOWN 8 taps over output voxels, UP 8 taps over input voxels
    c = C0
    L = [("c", 16, c, 0), ("c", c, c, 0), ("d", c, 2 * c, 1), ("c", 2 * c, 2 * c, 1), ("c", 2 * c, 2 * c, 1),
         ("d", 2 * c, 4 * c, 2), ("c", 4 * c, 4 * c, 2), ("c", 4 * c, 4 * c, 2), ("d", 4 * c, 8 * c, 3),
         ("c", 8 * c, 8 * c, 3), ("c", 8 * c, 8 * c, 3), ("u", 8 * c, 4 * c, 3), ("c", 8 * c, 4 * c, 2),
         ("c", 4 * c, 4 * c, 2), ("u", 4 * c, 2 * c, 2), ("c", 4 * c, 2 * c, 1), ("c", 2 * c, 2 * c, 1),
         ("u", 2 * c, c, 1), ("c", 2 * c, c, 0), ("c", c, c, 0)]
    fwd = []
    for mode, ci, co, lev in L:
        rows = N * (D >> lev) ** 3
        fwd.append(2.0 * rows * (27 if mode == "c" else 8) * ci * co)
    f = sum(fwd)
    return {"forward": f, "train_step": 3.0 * f - fwd[0]}


def bench_surrogate(args):
    """Training steps of the warm-start network (BF16 MFMA kernels, FP32
    accumulation, Adam) on a batch of N = 8 random 64^3 samples."""
    import torch

    from paper_1112_1071_amd import mcrt

    N, D = 8, 64
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn((N * D ** 3, 3), generator=g, device="cuda") * 2.0
    x[:, 1] -= 25.0
    x[:, 2] += 4.0
    y = torch.randn(N * D ** 3, generator=g, device="cuda") * 0.3 + 1.5
    k = torch.ones(N * D ** 3, device="cuda")
    sur = mcrt.Surrogate(0, 16, seed=1)
    for _ in range(args.warmup):
        sur.train_step(x, y, k, N, D, lr=1e-4, mask_count=float(N * D ** 3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sur.train_step(x, y, k, N, D, lr=1e-4, mask_count=float(N * D ** 3))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    t1 = time.perf_counter()
    for _ in range(args.steps):
        sur.forward(x, N, D)
    torch.cuda.synchronize()
    ms_fwd = (time.perf_counter() - t1) * 1e3 / args.steps
    fl = surrogate_flops(N, D)
    tf = fl["train_step"] / (ms * 1e-3) / 1e12
    out = {
        "metric": "warm-start network training steps per second (8 x 64^3 samples)",
        "value": 1e3 / ms, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "warm-start network: 4-level 3-D conv encoder-decoder, 16 base channels, "
                               "batch 8 x 64^3, forward + backward + Adam", "batch": N, "side": D},
        "roofline": {"bound": "mfma", "kernel": "whole training step", "achieved": tf,
                     "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / BF16_PEAK_TFLOPS,
                     "traffic": None, "flops_per_step": fl["train_step"]},
        "forward": {"ms": ms_fwd, "tflops": fl["forward"] / (ms_fwd * 1e-3) / 1e12},
    }
    print(json.dumps(out), flush=True)


def warmstart_runs(family: str, count: int, packets: float, ppc: float, weights: str) -> dict:
    """Time to a converged temperature (max dT/T < 1 % over the noise mask),
    from T = 10 K and from the learned warm start, on `count` unseen models:
    128^3 clumps built like the 256^3 clump, or thick disks of the training
    family's holdout; the warm-start time includes feature computation and
    network inference."""
    from paper_1112_1071_amd import mcrt, warmstart

    sur = mcrt.Surrogate(0, 16, seed=0)
    sur.load(weights)
    runs = []
    if family == "disk":
        cfgs = warmstart.thick_holdout_disks(count, packets_per_cell=ppc)
        n_packets = int(cfgs[0]["run"]["n_packets"])
        workload = (f"{count} thick holdout disks of the training family (64^3, mid-plane "
                    f"tau(1 um) >= {warmstart.THICK_DISK_TAU:g}), {ppc:g} packets per cell per iteration")
    else:
        cfgs = [warmstart.test_clump(i, n_packets=int(packets)) for i in range(count)]
        n_packets = int(packets)
        workload = (f"{count} unseen 128^3 clumps built like the 256^3 clump (0.65 pc, "
                    f"50 sources, mean tau(1 um) 50), {packets:.2e} packets per iteration")
    for i, cfg in enumerate(cfgs):
        cold = warmstart.converge(cfg, None)
        warm = warmstart.converge(cfg, sur)
        runs.append({"model": i, "cold": cold, "warm": warm})
        print(f"# {family} {i}: cold {cold['iterations']} it {cold['ms_to_converged'] or -1:.0f} ms, "
              f"warm {warm['iterations']} it {warm['ms_to_converged'] or -1:.0f} ms, pre-MC median "
              f"|dlnT| {warm['pre_mc_error']['median_abs_dlnT']:.3f}", file=sys.stderr, flush=True)
    ok = all(r["cold"]["converged"] and r["warm"]["converged"] for r in runs)
    t_cold = float(np.mean([r["cold"]["ms_to_converged"] or np.nan for r in runs]))
    t_warm = float(np.mean([r["warm"]["ms_to_converged"] or np.nan for r in runs]))
    return {
        "workload": workload, "models": count, "packets_per_iteration": n_packets,
        "cold": {"ms_to_converged": t_cold, "iterations": [r["cold"]["iterations"] for r in runs]},
        "warm": {"ms_to_converged": t_warm, "iterations": [r["warm"]["iterations"] for r in runs],
                 "ms_inference": [r["warm"]["ms_warm_start"] for r in runs],
                 "pre_mc_error": [r["warm"]["pre_mc_error"] for r in runs]},
        "speedup": t_cold / t_warm if ok else None, "all_converged": ok,
    }


def bench_warmstart(args):
    w = warmstart_runs(args.family, args.clumps, args.packets, args.ppc, args.weights)
    out = {
        "metric": "time to converged T (max dT/T < 1%), learned warm start",
        "value": w["warm"]["ms_to_converged"], "unit": "ms", "n_gpus": 1, "steps": w["models"],
        "warmup": 0, "ms_per_step": w["warm"]["ms_to_converged"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32 transport, bf16 network",
        "data": "synthetic",
        "config": {"workload": w["workload"], "models": w["models"],
                   "packets_per_step": w["packets_per_iteration"]},
        "cold": w["cold"], "warm": w["warm"], "speedup": w["speedup"],
        "all_converged": w["all_converged"],
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["clump256", "sphere32", "disk128", "batch", "warmstart", "raytrace",
                                           "surrogate", "pda"], default="clump256")
    ap.add_argument("--npix", type=int, default=256, help="raytrace: image pixels per side")
    ap.add_argument("--clumps", type=int, default=2, help="warmstart: test models")
    ap.add_argument("--family", choices=["clump", "disk"], default="clump",
                    help="warmstart: unseen 128^3 clumps or thick holdout disks (64^3)")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1112_1071_amd", "weights",
                                                      "warmstart_c16.npy"))
    ap.add_argument("--models", type=int, default=512)
    ap.add_argument("--ppc", type=int, default=0,
                    help="packets per cell per iteration (batch: default 30; warmstart disks: 400)")
    ap.add_argument("--seq-models", type=int, default=512)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=float, default=1e8)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default=None,
                    help="transport precision (default: fp64 for sphere32, fp32 otherwise)")
    ap.add_argument("--cpu-packets", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-warmstart", action="store_true",
                    help="skip the warm-start vs cold-start runs of the default line")
    ap.add_argument("--defer", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--walk-batch", type=int, default=0)
    ap.add_argument("--layout", type=int, default=-1)
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--sampling", type=int, default=0, help="1: equal packets per source")
    ap.add_argument("--mode", type=int, default=-1,
                    help="transport_mode: 0 per-lane persistent walk, 1 tiled sweeps")
    ap.add_argument("--tile-z", type=int, default=0)
    ap.add_argument("--tile-xy", type=int, default=0)
    ap.add_argument("--tally-copies", type=int, default=0)
    ap.add_argument("--visit-events", type=int, default=0)
    ap.add_argument("--sweep-batch", type=int, default=0,
                    help="tiled sweeps: packets emitted at a time (0: default 2^25)")
    ap.add_argument("--drain", type=int, default=0,
                    help="tiled sweeps: records left for the per-lane finish (-1 never, 0 default)")
    ap.add_argument("--mrw", type=float, default=0.0, help="modified random walk gamma (0 = off)")
    ap.add_argument("--max-events", type=int, default=0, help="batch: interactions before a kill")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batch":
        args.ppc = args.ppc or 30
        bench_batch(args)
        return
    if args.workload == "raytrace":
        bench_raytrace(args)
        return
    if args.workload == "surrogate":
        bench_surrogate(args)
        return
    if args.workload == "pda":
        bench_pda(args)
        return
    if args.workload == "warmstart":
        if args.packets == 1e8:
            args.packets = 2.5e8
        args.ppc = args.ppc or 400
        bench_warmstart(args)
        return

    from paper_1112_1071_amd import mcrt, synth

    t0 = time.time()
    n_packets = int(args.packets)
    n_iter = args.warmup + args.steps
    if args.workload == "sphere32":
        # the small FP64 case: 32^3 sphere, one star, 100 bins, 1e5 packets
        n_packets = int(args.packets) if args.packets != 1e8 else 100_000
        cfg = synth.config0(n=32, n_packets=n_packets, n_iter=n_iter)
        what, cpu_n, cpu_1 = "32^3 sphere", n_packets, n_packets
        workload = (f"sphere32: 32^3 uniform sphere (tau(1 um) = 1), 5800 K star, 100 frequency bins, "
                    f"{n_packets:.0e} packets per Lucy iteration")
        prec_default = "fp64"
        mode_default = 0
    elif args.workload == "disk128":
        # the flared disk: 128^3, mid-plane tau(1 um) = 1e3, 200 bins, 1e7 packets
        n_packets = int(args.packets) if args.packets != 1e8 else 10_000_000
        cfg = synth.config1(n=128, n_packets=n_packets, n_iter=n_iter)
        what, cpu_n, cpu_1 = "128^3 disk", 2_000_000, 200_000
        workload = (f"disk128: 128^3 flared disk (mid-plane tau(1 um) = 1e3), 4000 K star, 200 frequency "
                    f"bins, {n_packets:.0e} packets per Lucy iteration")
        prec_default = "fp32"
        mode_default = 0
    else:
        cfg = synth.config2(n=args.grid, n_packets=n_packets, n_iter=n_iter)
        what, cpu_n, cpu_1 = f"{args.grid}^3 clump", args.cpu_packets, 200_000
        workload = (f"clump{args.grid}: {args.grid}^3 log-normal star-forming clump, 50 point "
                    f"sources, 200 frequency bins, {n_packets:.0e} packets per Lucy iteration")
        prec_default = "fp32"
        mode_default = -1
    gen_s = time.time() - t0
    precision = args.precision or prec_default
    prec = mcrt.MCRT_FP32_TRANSPORT if precision == "fp32" else mcrt.MCRT_FP64
    run = dict(precision=prec)
    if args.defer:
        run["defer_lanes"] = args.defer
    if args.blocks_per_cu:
        run["blocks_per_cu"] = args.blocks_per_cu
    if args.walk_batch:
        run["walk_batch"] = args.walk_batch
    if args.layout >= 0:
        run["grid_layout"] = args.layout
    if args.block_size:
        run["block_size"] = args.block_size
    if args.sampling:
        run["source_sampling"] = args.sampling
    if args.mrw > 0:
        run["mrw_gamma"] = args.mrw
    # the per-lane walk is the faster transport on the small sphere (6.8x) and
    # on the mostly empty disk (1.7x); the tiled sweeps on the dense clumps
    mode = args.mode if args.mode >= 0 else mode_default
    if mode >= 0:
        run["transport_mode"] = mode
    if args.tile_z:
        run["tile_z"] = args.tile_z
    if args.tile_xy:
        run["tile_xy"] = args.tile_xy
    if args.tally_copies:
        run["tally_copies"] = args.tally_copies
    if args.visit_events:
        run["visit_events"] = args.visit_events
    if args.drain:
        run["sweep_drain"] = args.drain
    if args.sweep_batch:
        run["sweep_batch"] = args.sweep_batch
    model = mcrt.Model(cfg, **run)
    print(f"# workload built in {gen_s:.1f} s; warmup {args.warmup}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        st = model.iterate()
        print(f"# warmup {i}: {st['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    import torch

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    stats = []
    for i in range(args.steps):
        st = model.iterate()
        stats.append(st)
        print(f"# step {i}: {st['ms_total']:.1f} ms (transport {st['ms_transport']:.1f} ms)",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = 1e3 * elapsed / args.steps
    value = n_packets * args.steps / elapsed
    # every step transported every packet to an escape or a kill, and conserved
    # the sources' energy (immediate re-emission, Sec. 1; dt = 1 s)
    L = sum(float(s["lum"]) for s in cfg["sources"])
    for i, st in enumerate(stats):
        if st["n_escape"] + st["n_killed"] != n_packets:
            raise SystemExit(f"step {i}: {st['n_escape']} escaped + {st['n_killed']} killed != {n_packets}")
        if abs(st["e_escaped"] + st["e_killed"] - L) > 1e-9 * L:
            raise SystemExit(f"step {i}: escaped + killed energy {st['e_escaped'] + st['e_killed']} != L {L}")

    ms_tr = float(np.mean([s["ms_transport"] for s in stats]))
    # the dominant kernel (the sweep kernel of the tiled transport, summed over
    # its launches of a pass; the one launch of the per-lane walk), timed by
    # HIP events on the stream it runs on
    ms_dom = float(np.mean([s["ms_dominant"] for s in stats]))
    # launches of the dominant kernel: the sweeps, plus the per-lane finish of
    # the tail when the pass used it
    launches = (float(np.mean([s["n_sweeps"] + (1 if s["n_drained"] else 0) for s in stats]))
                if model.run["transport_mode"] == 1 else 1.0)
    abytes = float(np.mean([algorithmic_bytes(s, prec) for s in stats]))
    achieved = abytes / (ms_dom * 1e-3) / 1e9
    traffic_dom, traffic_pass = measured_traffic(prec, int(model.run["transport_mode"]), args.workload)
    # counter bytes of the dominant kernel per pass over the launches timed
    # here, the same division as the algorithmic bytes
    traffic = traffic_dom / launches if traffic_dom else None
    last = stats[-1]
    out = {
        "metric": f"packets/s at {int(cfg['grid']['n'][0])}^3 (Lucy iterations)",
        "value": value,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32" if prec == 1 else "fp64",
        "data": "synthetic",
        "config": {
            "workload": f"{workload}, {'FP32' if prec == 1 else 'FP64'} transport with FP64 reductions",
            "grid": int(cfg["grid"]["n"][0]), "packets_per_step": n_packets, "precision": precision,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_sweep (+ k_sweep_drain)" if model.run["transport_mode"] == 1 else "k_transport",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            # per launch of the dominant kernel (launches: the sweeps of a pass)
            "algorithmic_bytes_per_launch": abytes / launches,
            "ms_per_launch": ms_dom / launches,
            "launches_per_pass": launches,
            # the same algorithmic bytes over the whole pass (every transport
            # kernel: emission, scans, grouping and sweeps)
            "pass_GBs": abytes / (ms_tr * 1e-3) / 1e9,
            "ms_pass": ms_tr,
            # HBM bytes the counters measured per launch of the dominant kernel,
            # over its launch time, and for the whole pass (null unless taken
            # on the current sources)
            "hbm_measured_GBs": traffic / (ms_dom / launches * 1e-3) / 1e9 if traffic else None,
            "traffic_pass": traffic_pass,
        },
        "detail": {
            "crossings_per_s": (last["n_cross_dust"] + last["n_cross_empty"]) / (last["ms_transport"] * 1e-3),
            "dust_crossings": last["n_cross_dust"], "empty_crossings": last["n_cross_empty"],
            "scatters": last["n_scatter"], "absorptions": last["n_absorb"],
            "killed": last["n_killed"], "ms_update": last["ms_update"],
            "transport_mode": model.run["transport_mode"], "sweeps": last["n_sweeps"],
            "tile_visits": last["n_visits"], "drained_records": last["n_drained"],
            "max_dT": last["max_dT"], "q": last["q"],
        },
    }
    model.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, cpu_n, what, cpu_1)
        out["cpu_baseline"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    if not args.no_warmstart and args.workload == "clump256":
        # the metric's second half: time to a converged T, warm start vs cold
        # start, on one unseen 128^3 clump and one thick holdout disk
        del cfg
        out["warmstart"] = {
            "clump128": warmstart_runs("clump", 1, 2.5e8, 0, args.weights),
            "disk64": warmstart_runs("disk", 1, 0, 400, args.weights),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
