"""Form 2 (batching): many uneven models in one persistent launch per Lucy
iteration, replayed from a hipGraph, launch shape autotuned.  Each model's
results must equal its own single-model run (same seed) up to FP64 summation
order, and the oracle's for a sample of models."""
import numpy as np
import pytest

import oracle
from paper_1112_1071_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    from paper_1112_1071_amd import mcrt

    mcrt.lib()
    return mcrt


def small_family(n_models, packets_per_cell=3, n_min=8, n_max=20):
    return [synth.config3_model(m, packets_per_cell=packets_per_cell, n_iter=3, n_min=n_min,
                                n_max=n_max) for m in range(n_models)]


@pytest.mark.parametrize("graph", [0, 1])
def test_batch_equals_single_model_runs(M, graph):
    cfgs = small_family(12)
    run = dict(precision=M.MCRT_FP64)
    batch = [M.Model(c, **run) for c in cfgs]
    solo = [M.Model(c, **run) for c in cfgs]
    st = M.batch_run(batch, n_iter=3, final_pass=1, use_graph=graph, autotune=0)
    assert st["n_iterations"] == 3 and st["graph_used"] == graph
    for b, s, c in zip(batch, solo, cfgs):
        for _ in range(3):
            s.iterate()
        s.final_pass()
        ab, as_ = b.specific_energy(), s.specific_energy()
        nz = as_ > 0
        assert np.array_equal(nz, ab > 0), c["name"]
        assert np.max(np.abs(ab[nz] / as_[nz] - 1)) < 1e-9, c["name"]
        assert np.max(np.abs(b.temperature() / s.temperature() - 1)) < 1e-9, c["name"]
        sb, ss = b.sed(), s.sed()
        assert np.array_equal(sb[2], ss[2]), c["name"]
        assert np.allclose(sb[0], ss[0], rtol=1e-12, atol=0), c["name"]


def test_batch_fp32_equals_single_model_runs(M):
    # FP32 transport: the batched launch and one per-lane-walk launch per
    # model follow the same packets; the FP64 tallies differ only in
    # summation order
    cfgs = small_family(12)
    run = dict(precision=M.MCRT_FP32_TRANSPORT, transport_mode=0)
    batch = [M.Model(c, **run) for c in cfgs]
    solo = [M.Model(c, **run) for c in cfgs]
    st = M.batch_run(batch, n_iter=1, final_pass=0, use_graph=0, autotune=0)
    assert st["block_size"] == 256
    for b, s, c in zip(batch, solo, cfgs):
        s.iterate()
        ab, as_ = b.specific_energy(), s.specific_energy()
        nz = as_ > 0
        assert np.array_equal(nz, ab > 0), c["name"]
        assert np.max(np.abs(ab[nz] / as_[nz] - 1)) < 1e-9, c["name"]
        assert np.max(np.abs(b.temperature() / s.temperature() - 1)) < 1e-9, c["name"]


def test_batch_sample_against_oracle(M):
    cfgs = small_family(6)
    batch = [M.Model(c, precision=M.MCRT_FP64) for c in cfgs]
    M.batch_run(batch, n_iter=2, final_pass=0, use_graph=1, autotune=0)
    for b, c in list(zip(batch, cfgs))[:3]:
        o = oracle.OracleModel(c)
        o.iterate()
        o.iterate()
        ao, ab = o.specific_energy(), b.specific_energy()
        nz = ao > 0
        assert np.array_equal(nz, ab > 0)
        assert np.max(np.abs(ab[nz] / ao[nz] - 1)) < 1e-9
        assert np.max(np.abs(b.temperature() / o.temperature() - 1)) < 1e-8


def test_batch_autotune_and_cache(M):
    cfgs = small_family(8, packets_per_cell=2)
    for expect in (1, 2):
        batch = [M.Model(c, precision=M.MCRT_FP32_TRANSPORT) for c in cfgs]
        st = M.batch_run(batch, n_iter=1, final_pass=0, autotune=1, tune_fraction=0.2)
        assert st["tuned"] == expect
        assert st["block_size"] in (128, 256) and st["walk_batch"] in (2, 4, 8)
        L = [sum(s["lum"] for s in c["sources"]) for c in cfgs]
        for b, l in zip(batch, L):
            T = b.temperature()
            assert np.all(np.isfinite(T)) and T.min() >= 1.0


def test_batch_rejects_mixed_precision(M):
    cfgs = small_family(2)
    a = M.Model(cfgs[0], precision=M.MCRT_FP64)
    b = M.Model(cfgs[1], precision=M.MCRT_FP32_TRANSPORT)
    with pytest.raises(M.MCRTError):
        M.batch_run([a, b], n_iter=1, autotune=0)
