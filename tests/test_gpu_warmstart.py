"""What the trained warm-start network gains over the plain method.

The committed network (paper_1112_1071_amd/weights/warmstart_c16.npy, trained
by paper_1112_1071_amd/warmstart.py on Monte-Carlo temperature fields of the
training family) starts the Lucy iteration of an unseen clump.  Against the
plain start (T = 10 K everywhere) it must
  * predict the converged temperatures far better before any Monte-Carlo
    iteration (median |ln T0/T_conv| over dust cells),
  * leave the first Monte-Carlo iteration closer to the converged field,
  * need no more iterations to meet max dT/T < 1 % over the noise mask.
The converged field is a long cold run of the same clump.
"""
import os

import numpy as np
import pytest

from paper_1112_1071_amd import synth, warmstart

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(warmstart.__file__), "weights", "warmstart_c16.npy")


@pytest.fixture(scope="module")
def M():
    from paper_1112_1071_amd import mcrt

    mcrt.lib()
    return mcrt


def _clump():
    # an unseen clump with the test recipe at the training resolution: 64^3
    # cells of the 128^3 test clumps' size, 12 sources
    return synth.config2(n=64, n_packets=12_000_000, n_iter=8, seed=45077, gen_seed=45077, n_src=12,
                         box=0.65 * synth.PC / 2)


def test_warm_start_beats_cold_start(M):
    cfg = _clump()
    sur = M.Surrogate(0, 16, seed=0)
    sur.load(WEIGHTS)
    rho = np.asarray(cfg["rho"]).reshape(-1)
    # reference: cold run to convergence
    ref = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT)
    for _ in range(6):
        ref.iterate()
    T_conv = ref.temperature()
    dust = (rho > 0) & (T_conv > 1.0)

    def err(T):
        return float(np.median(np.abs(np.log(T[dust] / T_conv[dust]))))

    warm = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, want_noise=1, stop_on_convergence=1,
                   n_packets_final=1000)
    warm.warm_start(sur)
    T0_warm = warm.temperature()
    cold = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, want_noise=1, stop_on_convergence=1,
                   n_packets_final=1000)
    e_warm0, e_cold0 = err(T0_warm), err(np.full(rho.size, 10.0))
    print(f"pre-MC median |dlnT|: warm {e_warm0:.4f}, cold {e_cold0:.4f}")
    assert e_warm0 < 0.5 * e_cold0

    warm.iterate()
    cold.iterate()
    e_warm1, e_cold1 = err(warm.temperature()), err(cold.temperature())
    print(f"after one iteration: warm {e_warm1:.4f}, cold {e_cold1:.4f}")
    assert e_warm1 < e_cold1

    rw = warm.run_all()
    rc = cold.run_all()
    it_w = 1 + rw["n_iterations"]
    it_c = 1 + rc["n_iterations"]
    print(f"iterations to max dT/T < 1%: warm {it_w}, cold {it_c}")
    assert rw["converged"] and rc["converged"]
    assert it_w <= it_c
    sur.close()
