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


def test_traffic_per_sweep_launch_and_per_pass(tmp_path):
    sweep = "void mcrt::k_sweep<float, false, false>(mcrt::SweepParams)"
    emit = "void mcrt::k_sweep_emit<float, false>(mcrt::SweepParams)"
    other = "void (anonymous namespace)::k_update(Foo)"
    # two sweeps (100 and 300 KiB read), one emission (50), one unrelated kernel
    _write(tmp_path / "f", [(1, sweep, "FETCH_SIZE", 100), (2, sweep, "FETCH_SIZE", 300),
                            (3, emit, "FETCH_SIZE", 50), (4, other, "FETCH_SIZE", 1e6)])
    _write(tmp_path / "w", [(1, sweep, "WRITE_SIZE", 10), (2, sweep, "WRITE_SIZE", 30),
                            (3, emit, "WRITE_SIZE", 5), (4, other, "WRITE_SIZE", 1e6)])
    # the copy moves 1 GiB: FETCH reads half of it, WRITE all of it
    copy = "void copyBuffer(...)"
    _write(tmp_path / "cf", [(1, copy, "FETCH_SIZE", (1 << 30) / 2)])
    _write(tmp_path / "cw", [(1, copy, "WRITE_SIZE", 1 << 30)])
    a = SimpleNamespace(fetch=str(tmp_path / "f"), write=str(tmp_path / "w"),
                        copy_fetch=str(tmp_path / "cf"), copy_write=str(tmp_path / "cw"),
                        iterations=1, precision=1, mode=1, workload="clump256")
    r = profiling.traffic(a)
    assert r["fetch_scale"] == pytest.approx(2.0) and r["write_scale"] == pytest.approx(1.0)
    assert r["launches"] == 2
    assert r["fetch_bytes_per_launch"] == pytest.approx(2.0 * 200)
    assert r["write_bytes_per_launch"] == pytest.approx(20)
    assert r["hbm_bytes_per_launch"] == pytest.approx(420)
    # the pass sums every transport kernel (sweeps and emission), not k_update
    assert r["fetch_bytes_per_pass"] == pytest.approx(2.0 * 450)
    assert r["write_bytes_per_pass"] == pytest.approx(45)
