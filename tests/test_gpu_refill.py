"""The tiled transport's pool refill and tail (Sec. 2.2 packets, Eq. 2 tallies), driven
with a small emission batch so that one pass refills the pool many times: the
path the 1e8-packet benchmark pass takes with its 2^25-packet batches.

Every packet's history is independent of when it was emitted and of which
sweep walks it (its random stream is keyed by its id), so

* FP64, same stream: the event sequences of the first packets, all counters
  and the per-cell absorption tally equal the oracle's (tallies to the
  summation order, 1e-9), for several batch sizes;
* FP32 in the benchmark's launch shape: the counters are identical whatever
  the batch, and the per-cell tallies agree with the run without refills and
  with the per-lane walk to FP64 summation order (every side adds the same
  FP32 products into FP64 sums: 1e-9);
* both: energy is conserved, escaped + killed = L dt, and every packet ends
  as an escape or a kill.
"""
import numpy as np
import pytest

import oracle
from paper_1112_1071_amd import synth

pytestmark = pytest.mark.gpu

COUNTERS = ["n_cross_dust", "n_cross_empty", "n_scatter", "n_absorb", "n_escape", "n_killed"]


@pytest.fixture(scope="module")
def M():
    from paper_1112_1071_amd import mcrt

    mcrt.lib()
    return mcrt


def _logs_equal(eo, co, eg, cg):
    assert np.array_equal(co, cg), f"event counts differ for {np.sum(co != cg)} packets"
    cap = eo.shape[1]
    idx = np.arange(cap)[None, :] < np.minimum(co, cap)[:, None]
    for f in ["type", "nu", "incl"]:
        assert np.array_equal(eo[f][idx], eg[f][idx]), f
    assert np.array_equal(eo["cell"][idx], eg["cell"][idx])


@pytest.fixture(scope="module")
def sphere_oracle():
    cfg = synth.config0(n=32, tau=2.0, n_packets=100_000, n_iter=1, n_bins=40)
    run = dict(event_log_packets=3000, event_log_cap=64)
    o = oracle.OracleModel(cfg, **run)
    so = o.iterate()
    eo, co = o.event_log()
    ao = o.specific_energy()
    o.close()
    return cfg, run, so, (eo, co), ao


@pytest.mark.parametrize("batch", [4096, 9999, 65536])
def test_fp64_refills_match_oracle(M, sphere_oracle, batch):
    cfg, run, so, (eo, co), ao = sphere_oracle
    g = M.Model(cfg, precision=M.MCRT_FP64, transport_mode=1, sweep_batch=batch, **run)
    sg = g.iterate()
    for k in COUNTERS:
        assert sg[k] == so[k], (k, sg[k], so[k])
    eg, cg = g.event_log()
    _logs_equal(eo, co, eg, cg)
    ag = g.specific_energy()
    nz = ao > 0
    assert np.array_equal(nz, ag > 0)
    np.testing.assert_allclose(ag[nz], ao[nz], rtol=1e-9)
    L = sum(s["lum"] for s in cfg["sources"])
    assert sg["e_escaped"] + sg["e_killed"] == pytest.approx(L, rel=1e-12)
    assert sg["n_escape"] + sg["n_killed"] == 100_000
    # a pass of 1e5 packets in batches of `batch` sweeps more than once per batch
    assert sg["n_sweeps"] >= 100_000 // batch
    g.close()


def test_fp32_refills_in_benchmark_shape(M):
    # the benchmark's FP32 launch shape (24x24x20 tiles, 512 threads) on a
    # 64^3 clump with 20 sources; 2e5 packets in batches of 5000 (40 refills)
    cfg = synth.config2(n=64, n_packets=200_000, n_iter=1)
    ref = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, transport_mode=1)
    sr = ref.iterate()
    ar = ref.specific_energy()
    ref.close()
    assert sr["n_sweeps"] > 0
    for batch in (5000, 32768):
        g = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, transport_mode=1, sweep_batch=batch)
        sg = g.iterate()
        for k in COUNTERS:
            assert sg[k] == sr[k], (batch, k, sg[k], sr[k])
        ag = g.specific_energy()
        nz = ar > 0
        assert np.array_equal(nz, ag > 0)
        np.testing.assert_allclose(ag[nz], ar[nz], rtol=1e-9)
        L = sum(s["lum"] for s in cfg["sources"])
        assert sg["e_escaped"] + sg["e_killed"] == pytest.approx(L, rel=1e-9)
        assert sg["n_escape"] + sg["n_killed"] == 200_000
        g.close()


def test_fp32_tiled_refills_equal_the_per_lane_walk(M):
    # the same packets walked by the per-lane kernel (no tiles, no records):
    # identical counters, tallies to FP64 summation order
    cfg = synth.config2(n=64, n_packets=100_000, n_iter=1)
    a = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, transport_mode=0)
    b = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, transport_mode=1, sweep_batch=3000)
    sa, sb = a.iterate(), b.iterate()
    for k in COUNTERS:
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    aa, ab = a.specific_energy(), b.specific_energy()
    nz = aa > 0
    assert np.array_equal(nz, ab > 0)
    np.testing.assert_allclose(ab[nz], aa[nz], rtol=1e-9)
    a.close()
    b.close()


@pytest.mark.parametrize("drain", [-1, 1000, 1 << 30])
def test_fp64_tail_finish_matches_oracle(M, sphere_oracle, drain):
    # once every packet is emitted and at most `drain` records remain, the
    # per-lane walk finishes them (-1: never; 2^30: everything left after the
    # emission): the same histories as the oracle's either way
    cfg, run, so, (eo, co), ao = sphere_oracle
    g = M.Model(cfg, precision=M.MCRT_FP64, transport_mode=1, sweep_batch=9999, sweep_drain=drain, **run)
    sg = g.iterate()
    for k in COUNTERS:
        assert sg[k] == so[k], (drain, k, sg[k], so[k])
    eg, cg = g.event_log()
    _logs_equal(eo, co, eg, cg)
    ag = g.specific_energy()
    nz = ao > 0
    assert np.array_equal(nz, ag > 0)
    np.testing.assert_allclose(ag[nz], ao[nz], rtol=1e-9)
    if drain < 0:
        assert sg["n_drained"] == 0
    else:
        assert sg["n_drained"] > 0
    g.close()


def test_fp32_tail_finish_equals_sweeps(M):
    # the benchmark's FP32 launch shape with and without the per-lane finish
    cfg = synth.config2(n=64, n_packets=200_000, n_iter=1)
    a = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, transport_mode=1, sweep_drain=-1)
    b = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, transport_mode=1, sweep_drain=1 << 30)
    sa, sb = a.iterate(), b.iterate()
    assert sa["n_drained"] == 0 and sb["n_drained"] > 0
    for k in COUNTERS:
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    aa, ab = a.specific_energy(), b.specific_energy()
    nz = aa > 0
    assert np.array_equal(nz, ab > 0)
    np.testing.assert_allclose(ab[nz], aa[nz], rtol=1e-9)
    a.close()
    b.close()
