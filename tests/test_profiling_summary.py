"""Host logic of the rocprofv3 summaries: the counter runs are scaled by a
plain copy's reading and split per dispatch of the dominant kernel."""
import csv
import os
from types import SimpleNamespace

import pytest

from paper_1112_1071_amd import profiling

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_traffic_of_sweeps_and_tail_finish_per_pass(tmp_path):
    sweep = "void mcrt::k_sweep<float, false, false>(mcrt::SweepParams)"
    drain = "void mcrt::k_sweep_drain<float>(mcrt::SweepParams)"
    emit = "void mcrt::k_sweep_emit<float, false>(mcrt::SweepParams)"
    upd = "void (anonymous namespace)::k_update(Foo)"
    # two passes, each ended by its cell update (1e6 KiB, not transport):
    # pass 0: one sweep (500 KiB read), the emission (60); pass 1: two sweeps
    # (100, 300), the tail's finish (20), the emission (50)
    fr = [(1, emit, 60), (2, sweep, 500), (3, upd, 1e6),
          (4, emit, 50), (5, sweep, 100), (6, sweep, 300), (7, drain, 20), (8, upd, 1e6)]
    # listed out of dispatch order: the passes follow the dispatch ids
    _write(tmp_path / "f", [(i, k, "FETCH_SIZE", v) for i, k, v in reversed(fr)])
    _write(tmp_path / "w", [(i, k, "WRITE_SIZE", v / 10) for i, k, v in fr])
    # the copy moves 1 GiB: FETCH reads half of it, WRITE all of it
    copy = "void copyBuffer(...)"
    _write(tmp_path / "cf", [(1, copy, "FETCH_SIZE", (1 << 30) / 2)])
    _write(tmp_path / "cw", [(1, copy, "WRITE_SIZE", 1 << 30)])
    a = SimpleNamespace(fetch=str(tmp_path / "f"), write=str(tmp_path / "w"),
                        copy_fetch=str(tmp_path / "cf"), copy_write=str(tmp_path / "cw"),
                        iterations=1, skip=1, precision=1, mode=1, workload="clump256")
    r = profiling.traffic(a)
    assert r["fetch_scale"] == pytest.approx(2.0) and r["write_scale"] == pytest.approx(1.0)
    # the second pass alone: sweeps and the tail's finish, not the emission
    assert r["dispatches_per_pass"] == 3
    assert r["dominant_fetch_bytes_per_pass"] == pytest.approx(2.0 * 420)
    assert r["dominant_write_bytes_per_pass"] == pytest.approx(42)
    assert r["dominant_bytes_per_pass"] == pytest.approx(882)
    # every transport kernel of the pass (sweeps, finish, emission), not k_update
    assert r["fetch_bytes_per_pass"] == pytest.approx(2.0 * 470)
    assert r["write_bytes_per_pass"] == pytest.approx(47)
    # both passes, averaged
    a.skip, a.iterations = 0, 2
    r = profiling.traffic(a)
    assert r["dispatches_per_pass"] == 2
    assert r["dominant_fetch_bytes_per_pass"] == pytest.approx(2.0 * 920 / 2)
    assert r["fetch_bytes_per_pass"] == pytest.approx(2.0 * 1030 / 2)


def test_iterations_split_with_several_counters_per_dispatch(tmp_path):
    # a run with two counters writes two rows per dispatch; the iteration ends
    # after both rows of its cell update
    sweep = "void mcrt::k_sweep<float, false, false>(mcrt::SweepParams)"
    upd = "void (anonymous namespace)::k_update(Foo)"
    fr = [(1, sweep, 5), (2, upd, 0), (3, sweep, 7), (4, upd, 0)]
    rows = [(i, k, c, v * (1 if c == "A" else 100)) for i, k, v in fr for c in ("A", "B")]
    _write(tmp_path / "p", rows)
    got = [(r["Dispatch_Id"], r["Counter_Name"]) for r in profiling._rows(str(tmp_path / "p"), 1, 1)]
    assert got == [("3", "A"), ("3", "B"), ("4", "A"), ("4", "B")]
    assert profiling._sum(str(tmp_path / "p"), "B", kernels=("k_sweep",), skip=0, iterations=1) == 500
