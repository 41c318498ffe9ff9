"""bench.py's command-line contract on the host: one GPU only (any other
count exits with a message and status 2), the argument parser, and the
algorithmic-bytes figure behind roofline.achieved."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_help_lists_the_workloads():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for w in ("clump256", "sphere32", "disk128", "batch", "warmstart", "raytrace", "surrogate", "pda"):
        assert w in r.stdout


def test_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import bench

    st = {"n_cross_dust": 10, "n_cross_empty": 3, "n_absorb": 2}
    # FP32: 4 B density + 16 B tally read-modify-write per dust segment, 4 B per
    # empty segment, 4 B emission-row position per absorption
    assert bench.algorithmic_bytes(st, 1) == 10 * 20 + 3 * 4 + 2 * 4
    # FP64: 8 B density and row position
    assert bench.algorithmic_bytes(st, 0) == 10 * 24 + 3 * 8 + 2 * 8


def test_surrogate_flops():
    sys.path.insert(0, ROOT)
    import bench

    one, two = bench.surrogate_flops(1, 64), bench.surrogate_flops(2, 64)
    assert two["forward"] == 2 * one["forward"]
    # the first layer: 64^3 output voxels x 27 taps x 16 (padded) x 16 channels
    first = 2.0 * 64 ** 3 * 27 * 16 * 16
    assert one["train_step"] == 3 * one["forward"] - first
    # the 64^3 level's four 3x3x3 convolutions (16->16, 16->16, 32->16, 16->16)
    # carry more than half of the forward FLOPs
    top = 2.0 * 64 ** 3 * 27 * 16 * (16 + 16 + 32 + 16)
    assert 0.5 < top / one["forward"] < 0.6
