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
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def transport_source_hash() -> str:
    h = hashlib.sha256()
    for f in ["mcrt_transport.hip", "mcrt_internal.h"]:
        with open(os.path.join(ROOT, "paper_1112_1071_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(st: dict, precision: int) -> float:
    """Bytes the method must move per launch: per dust-cell segment a density
    gather (4 B FP32 / 8 B FP64) and an FP64 read-modify-write of the cell's
    absorption tally (16 B); per empty-cell segment the density gather; per
    absorption the cell's emission-row position (4 B / 8 B)."""
    rb = 4 if precision == 1 else 8
    return (st["n_cross_dust"] * (rb + 16) + st["n_cross_empty"] * rb + st["n_absorb"] * rb)


def measured_traffic(precision: int):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, if it was taken on the current transport source."""
    p = os.path.join(ROOT, "profiles", "transport_clump256_pmc.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("source_hash") != transport_source_hash() or d.get("precision") != precision:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(cfg: dict, n_packets: int) -> dict:
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    o = oracle.OracleModel(cfg, n_threads=threads)
    st = o.transport_sample(n_packets)
    o.close()
    return {"value": n_packets / st["seconds"], "unit": "packets/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_packets} packets of a first Lucy iteration of the same 256^3 clump "
                      f"(FP64 oracle transport only, {st['seconds']:.1f} s)"}


def bench_batch(args):
    """Form 2: the batched family of uneven models, one persistent launch per
    Lucy iteration (graph-replayed, autotuned) vs one launch per model."""
    from paper_1112_1071_amd import mcrt, synth

    t0 = time.time()
    cfgs = [synth.config3_model(m, packets_per_cell=args.ppc, n_iter=args.steps)
            for m in range(args.models)]
    print(f"# {args.models} models built in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    prec = mcrt.MCRT_FP32_TRANSPORT if args.precision == "fp32" else mcrt.MCRT_FP64
    batch = [mcrt.Model(c, precision=prec) for c in cfgs]
    n_packets = sum(int(c["run"]["n_packets"]) for c in cfgs)
    cells = sum(int(np.prod(c["grid"]["n"])) for c in cfgs)
    # warm-up batch: tunes the launch shape (cached) and runs the first iteration
    stw = mcrt.batch_run(batch, n_iter=1, final_pass=0, use_graph=0, autotune=1)
    print(f"# warmup/tune: {stw['ms_total']:.0f} ms (tune {stw['ms_tune']:.0f} ms) shape "
          f"bs={stw['block_size']} K={stw['walk_batch']} defer={stw['defer_lanes']}",
          file=sys.stderr, flush=True)
    st = mcrt.batch_run(batch, n_iter=args.steps, final_pass=0, use_graph=1, autotune=1)
    ms_it = st["ms_iterations"] / st["n_iterations"]
    value = n_packets / (ms_it * 1e-3)
    print(f"# batched: {ms_it:.1f} ms per iteration", file=sys.stderr, flush=True)
    # the same iteration as one launch per model
    seq = [mcrt.Model(c, precision=prec) for c in cfgs[: args.seq_models]]
    for m in seq:
        m.iterate()
    import torch

    torch.cuda.synchronize()
    ts = time.perf_counter()
    for m in seq:
        m.iterate()
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - ts
    seq_packets = sum(int(c["run"]["n_packets"]) for c in cfgs[: args.seq_models])
    seq_value = seq_packets / seq_s
    out = {
        "metric": "packets/s, batched Lucy iterations of uneven models",
        "value": value, "unit": "packets/s", "n_gpus": 1, "steps": st["n_iterations"],
        "warmup": 1, "ms_per_step": ms_it, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32" if prec == 1 else "fp64", "data": "synthetic",
        "config": {"workload": f"batch{args.models}: {args.models} models, grids 16^3..96^3 "
                               f"({cells} cells), sphere/disk family, {args.ppc} packets per cell "
                               f"per iteration ({n_packets:.3e} packets)",
                   "models": args.models, "packets_per_step": n_packets},
        "batch": {"graph_used": st["graph_used"], "tuned": st["tuned"],
                  "block_size": st["block_size"], "walk_batch": st["walk_batch"],
                  "defer_lanes": st["defer_lanes"], "blocks_per_cu": st["blocks_per_cu"],
                  "ms_tune": stw["ms_tune"]},
        "sequential": {"value": seq_value, "unit": "packets/s", "models": args.seq_models,
                       "seconds": seq_s, "speedup_batched": value / seq_value},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["clump256", "batch"], default="clump256")
    ap.add_argument("--models", type=int, default=512)
    ap.add_argument("--ppc", type=int, default=30, help="batch: packets per cell per iteration")
    ap.add_argument("--seq-models", type=int, default=512)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=float, default=1e8)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--cpu-packets", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--defer", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--walk-batch", type=int, default=0)
    ap.add_argument("--layout", type=int, default=-1)
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--sampling", type=int, default=0, help="1: equal packets per source")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batch":
        bench_batch(args)
        return

    from paper_1112_1071_amd import mcrt, synth

    t0 = time.time()
    n_packets = int(args.packets)
    cfg = synth.config2(n=args.grid, n_packets=n_packets, n_iter=args.warmup + args.steps)
    gen_s = time.time() - t0
    prec = mcrt.MCRT_FP32_TRANSPORT if args.precision == "fp32" else mcrt.MCRT_FP64
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

    ms_tr = float(np.mean([s["ms_transport"] for s in stats]))
    abytes = float(np.mean([algorithmic_bytes(s, prec) for s in stats]))
    achieved = abytes / (ms_tr * 1e-3) / 1e9
    traffic = measured_traffic(prec)
    last = stats[-1]
    out = {
        "metric": "packets/s at 256^3 (Lucy iterations)",
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
            "workload": f"clump{args.grid}: {args.grid}^3 log-normal star-forming clump, 50 point "
                        f"sources, 200 frequency bins, {n_packets:.0e} packets per Lucy iteration, "
                        f"{'FP32' if prec == 1 else 'FP64'} transport with FP64 reductions",
            "grid": args.grid, "packets_per_step": n_packets, "precision": args.precision,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_transport",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": abytes,
            "ms_per_launch": ms_tr,
        },
        "detail": {
            "crossings_per_s": (last["n_cross_dust"] + last["n_cross_empty"]) / (last["ms_transport"] * 1e-3),
            "dust_crossings": last["n_cross_dust"], "empty_crossings": last["n_cross_empty"],
            "scatters": last["n_scatter"], "absorptions": last["n_absorb"],
            "killed": last["n_killed"], "ms_update": last["ms_update"],
            "max_dT": last["max_dT"], "q": last["q"],
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_packets)
        out["cpu_baseline"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
