"""Summaries of rocprofv3 output for the transport kernels.

    python -m paper_1112_1071_amd.profiling traffic --fetch DIR --write DIR \
        --copy-fetch DIR --copy-write DIR --iterations 2 --out FILE.json
    python -m paper_1112_1071_amd.profiling kernels --trace DIR --iterations 2 --out FILE.md
    python -m paper_1112_1071_amd.profiling copy     # the 1 GiB copy the counters are scaled by

`traffic` turns two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of the
benchmark into HBM bytes per transport pass.  Each counter is scaled by what
it reads for a plain 1 GiB device copy (bytes moved / counter), so that the
result is in bytes; the copy runs' directories give that factor.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
TRANSPORT_KERNELS = ("k_transport", "k_sweep", "k_refill_plan", "k_fill_u32")  # k_sweep* covers emit, scan, group
TRANSPORT_SOURCES = ("mcrt_transport.hip", "mcrt_sweep.hip", "mcrt_packet.h", "mcrt_internal.h", "mcrt_api.cpp")


def transport_source_hash() -> str:
    h = hashlib.sha256()
    for f in TRANSPORT_SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(d: str, skip: int = 0, iterations: int = 0):
    """counter rows in dispatch order; with `iterations` > 0, only those of the
    Lucy iterations skip .. skip + iterations - 1 (an iteration ends with its
    cell update, k_update)"""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    rows = [r for f in files for r in csv.DictReader(open(f))]
    if "Dispatch_Id" in (rows[0] if rows else {}):
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    # a dispatch has one row per counter: an iteration ends after the last
    # row of its k_update dispatch
    it, upd = 0, None
    for r in rows:
        did = r.get("Dispatch_Id")
        if upd is not None and did != upd:
            it, upd = it + 1, None
        if iterations <= 0 or skip <= it < skip + iterations:
            yield r
        if "k_update" in r["Kernel_Name"]:
            upd = did


def _sum(d: str, counter: str, kernels=TRANSPORT_KERNELS, skip: int = 0, iterations: int = 0) -> float:
    tot = 0.0
    for r in _rows(d, skip, iterations):
        if r["Counter_Name"] == counter and any(k in r["Kernel_Name"] for k in kernels):
            tot += float(r["Counter_Value"])
    return tot


def _copy_factor(d: str, counter: str) -> float:
    """bytes per counter unit from the copy runs: every copyBuffer dispatch
    moves 1 GiB one way (reads 1 GiB and writes 1 GiB)."""
    vals = [float(r["Counter_Value"]) for r in _rows(d)
            if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]]
    if not vals:
        raise ValueError(f"no copy dispatch in {d}")
    return (1 << 30) / (sum(vals) / len(vals))


def _dispatches(d: str, counter: str, names, skip: int = 0, iterations: int = 0):
    """(summed counter, number of dispatches) over the dispatches of the
    kernels named in `names` (each name followed by '<' in the kernel's name)"""
    per = defaultdict(float)
    pat = re.compile(r"(^|[\s:])(" + "|".join(re.escape(n) for n in names) + ")<")
    for r in _rows(d, skip, iterations):
        if r["Counter_Name"] == counter and pat.search(r["Kernel_Name"]):
            per[r.get("Dispatch_Id") or r.get("Correlation_Id")] += float(r["Counter_Value"])
    return sum(per.values()), len(per)


def traffic(a) -> dict:
    """HBM bytes per Lucy iteration of the dominant transport kernel (the
    sweeps and the per-lane finish of their tail, or the per-lane walk) and of
    every transport kernel.  The dominant kernel's bytes are given per pass:
    the device-driven sweep loop also launches a few sweeps that find no work,
    so a mean over dispatches would not be a mean over the launches that
    transport packets; the benchmark divides the per-pass figure by the
    launches it times (the sweeps that ran, plus the tail's finish)."""
    ff = _copy_factor(a.copy_fetch, "FETCH_SIZE")
    fw = _copy_factor(a.copy_write, "WRITE_SIZE")
    # the iterations skip .. skip + iterations - 1 of the run (skip 1 leaves
    # out the first pass, which starts from the initial temperature)
    sk = getattr(a, "skip", 0)
    fetch = _sum(a.fetch, "FETCH_SIZE", skip=sk, iterations=a.iterations) * ff / a.iterations
    write = _sum(a.write, "WRITE_SIZE", skip=sk, iterations=a.iterations) * fw / a.iterations
    dom = ("k_sweep", "k_sweep_drain") if a.mode == 1 else ("k_transport",)
    df, nf = _dispatches(a.fetch, "FETCH_SIZE", dom, sk, a.iterations)
    dw, nw = _dispatches(a.write, "WRITE_SIZE", dom, sk, a.iterations)
    if nf == 0 or nw == 0:
        raise ValueError(f"no {' / '.join(dom)} dispatch in the counter runs")
    return {"source_hash": transport_source_hash(), "precision": a.precision, "mode": a.mode,
            "workload": a.workload, "kernel": " + ".join(dom),
            "dominant_fetch_bytes_per_pass": df * ff / a.iterations,
            "dominant_write_bytes_per_pass": dw * fw / a.iterations,
            "dominant_bytes_per_pass": (df * ff + dw * fw) / a.iterations,
            "dispatches_per_pass": nf / a.iterations,
            "fetch_bytes_per_pass": fetch, "write_bytes_per_pass": write,
            "hbm_bytes_per_pass": fetch + write,
            "fetch_scale": ff, "write_scale": fw,
            "note": f"rocprofv3 FETCH_SIZE and WRITE_SIZE summed over the dispatches of "
                    f"{' and '.join(dom)} and over every transport kernel, per Lucy iteration "
                    f"(mean of {a.iterations} after skipping {sk}), scaled by a 1 GiB copy"}


def kernels(a) -> str:
    files = glob.glob(os.path.join(a.trace, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no kernel_stats.csv under {a.trace}")
    rows = list(csv.DictReader(open(files[0])))
    out = ["| kernel | calls | total ms | per iteration ms | average µs | % |", "|---|---|---|---|---|---|"]
    for r in rows[:12]:
        name = r["Name"].replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        tot = float(r["TotalDurationNs"]) / 1e6
        out.append(f"| `{name}` | {r['Calls']} | {tot:.1f} | {tot / a.iterations:.1f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)


def copy() -> None:
    """Two plain 1 GiB device-to-device copies (run under rocprofv3 --pmc to
    calibrate FETCH_SIZE and WRITE_SIZE)."""
    import torch

    n = 1 << 28
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {n * 4} bytes twice", flush=True)


def passes(trace_dir: str) -> str:
    """Per transport pass (the dispatches between two cell updates): summed
    durations of the transport kernels, of the dominant one, and the span from
    the first dispatch's start to the last one's end."""
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no kernel_trace.csv under {trace_dir}")
    rows = sorted(csv.DictReader(open(files[0])), key=lambda r: int(r["Start_Timestamp"]))
    out = ["| pass | dispatches | transport kernels ms | k_sweep / k_transport ms | span ms |",
           "|---|---|---|---|---|"]
    cur = []

    def flush():
        if not cur:
            return
        tot = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in cur) / 1e6
        dom = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in cur
                  if "k_sweep<" in r["Kernel_Name"] or "k_transport<" in r["Kernel_Name"]) / 1e6
        span = (int(cur[-1]["End_Timestamp"]) - int(cur[0]["Start_Timestamp"])) / 1e6
        out.append(f"| {len(out) - 2} | {len(cur)} | {tot:.1f} | {dom:.1f} | {span:.1f} |")

    for r in rows:
        name = r["Kernel_Name"]
        if "k_update" in name:
            flush()
            cur = []
        elif any(k in name for k in TRANSPORT_KERNELS):
            cur.append(r)
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--iterations", type=int, default=2)
    t.add_argument("--skip", type=int, default=0, help="Lucy iterations to leave out at the start")
    t.add_argument("--precision", type=int, default=1)
    t.add_argument("--mode", type=int, default=1)
    t.add_argument("--workload", default="clump256")
    t.add_argument("--out", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("--trace", required=True)
    k.add_argument("--iterations", type=int, default=3)
    k.add_argument("--out", required=True)
    sub.add_parser("copy")
    a = ap.parse_args()
    if a.cmd == "copy":
        copy()
    elif a.cmd == "traffic":
        res = traffic(a)
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res))
    else:
        txt = kernels(a) + "\n\n" + passes(a.trace)
        with open(a.out, "w") as f:
            f.write(txt + "\n")
        print(txt)
    return 0


if __name__ == "__main__":
    sys.exit(main())
