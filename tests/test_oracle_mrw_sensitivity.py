"""Why a few modified-random-walk histories part between two correct FP64
implementations (Sec. 2.2).

A walk step moves the packet to a random point of the sphere that touches
the nearest wall, and the next step's radius is the new distance to the
nearest wall: the map feeds a position's rounding back into the next radius,
so last-bit differences are carried and occasionally amplified over hundreds
of steps until a threshold decision (rho chi_R R0 >= gamma: step or plain
flight) comes out the other way.  The oracle shows this against itself: a
build that moves the point by one unit in the last place after every step
(ORC_MRW_NUDGE, test build only) parts from the plain build in a few packets
of the thick grey cube of the GPU walk tests, each time first at a step/no-
step decision after hundreds of steps, with the same counts otherwise.  The
GPU's FP64 walk (in-cell offsets, fused multiply-adds, its own sin/cos)
parts from the oracle at the same rate and in the same way, which is what
the GPU walk tests allow for."""
import ctypes as C
import os
import subprocess
import sys

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)


def _nudged_lib(tmp_path):
    out = str(tmp_path / "liborc_nudge.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-DORC_MRW_NUDGE", "-o", out,
                    os.path.join(os.path.dirname(oracle.__file__), "orc.c"), "-lm"], check=True)
    return out


def _logs(cfg):
    o = oracle.OracleModel(cfg, mrw_gamma=2.0, event_log_packets=2000, event_log_cap=16384)
    s = o.iterate()
    e, c = o.event_log()
    o.close()
    return s, e, c


def test_one_ulp_per_step_parts_few_histories(tmp_path, monkeypatch):
    from test_gpu_mrw import _thick_cube

    cfg = _thick_cube(True)
    s0, e0, c0 = _logs(cfg)
    # the same oracle with the nudge: swap the loaded library for the test build
    monkeypatch.setattr(oracle, "LIB_PATH", _nudged_lib(tmp_path))
    monkeypatch.setattr(oracle, "_lib", None)
    s1, e1, c1 = _logs(cfg)
    monkeypatch.setattr(oracle, "_lib", None)
    assert s0["n_mrw"] > 300_000
    parted = []
    for p in range(len(c0)):
        m = min(c0[p], c1[p], e0.shape[1])
        d = [np.flatnonzero(e0[f][p, :m] != e1[f][p, :m]) for f in ("type", "nu")]
        d = [x[0] for x in d if x.size]
        if d or c0[p] != c1[p]:
            parted.append((p, min(d) if d else m))
    print(f"{len(parted)} of {len(c0)} histories part after a one-ulp nudge per step", flush=True)
    assert 1 <= len(parted) <= 20
    for p, i in parted:
        # the first difference is a step on one side and a plain interaction on
        # the other, after hundreds of identical steps
        kinds = {int(e0["type"][p, i]), int(e1["type"][p, i])}
        assert oracle.EV_MRW in kinds
        assert np.sum(e0["type"][p, :i] == oracle.EV_MRW) >= 100
    # the aggregate result does not notice
    for k in ("n_scatter", "n_absorb", "n_escape"):
        assert abs(s0[k] - s1[k]) <= 1e-3 * s0[k]
