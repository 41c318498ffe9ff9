"""Modified random walk (Sec. 2.2) on the GPU against the FP64 oracle.

Same stream (FP64, same seed): the GPU takes the walk's steps at the same
points with the same draws, so counters, event sequences and the absorption
tally agree as for the plain walk.  The GPU reads the Planck- and
Rosseland-mean opacities from a table (cubic Hermite in ln T, ~1e-11), the
oracle evaluates them at T.  In thick cells a packet takes hundreds of
steps; a rare packet's history parts from the oracle's after thousands of
events, always first at a step/no-step decision (rho chi_R R0 >= gamma
decided the other way after hundreds of identical steps): in the grey
tau = 30 cube 6 of 2000 packets, in both transport modes, the same packets;
with power-law dust none.  The cause is the walk's own sensitivity, not the
table: each step's radius is the distance from the previous step's end point
to the nearest wall, so last-bit differences in position are carried and
occasionally amplified until a threshold decision flips.  The oracle parts
from itself in the same way (3 of 2000 packets after a one-ulp nudge per
step: test_oracle_mrw_sensitivity.py), and grey dust, where both sides use
the same opacity, shows it.  The bar: at least 99 % of the packets with identical event
sequences (98 % in the second iteration, at non-uniform temperatures),
counters to 1e-3, and Adot differences (the few parted packets cross most
cells of the small cube) well below those between two seeds of the oracle.
Both transport modes, grey and power-law dust.
"""
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


def _thick_cube(grey, n=4, tau_cell=30.0, n_packets=2000):
    cfg = synth.config0(n=n, n_packets=n_packets, n_iter=2, n_bins=20)
    if grey:
        nb = len(cfg["nu_edges"]) - 1
        cfg["dust"] = {"chi": np.full(nb, 100.0), "albedo": np.full(nb, 0.5), "g": np.zeros(nb)}
    chi1 = 100.0 if grey else 200.0  # power-law dust: chi(1 um) = 100 / (1 - 0.5)
    cfg["rho"][:] = tau_cell / (chi1 * 2 * synth.AU / n)
    if not grey:
        # warm dust: at 10 K the Rosseland mean of chi ~ nu^1 dust is far below
        # chi(1 um) and no cell would take a step
        cfg["run"]["t_init"] = 1500.0
    return cfg


@pytest.mark.parametrize("grey", [True, False])
@pytest.mark.parametrize("mode", [0, 1])
def test_mrw_same_stream(M, grey, mode):
    cfg = _thick_cube(grey)
    run = dict(mrw_gamma=2.0, event_log_packets=2000, event_log_cap=16384)
    o = oracle.OracleModel(cfg, **run)
    g = M.Model(cfg, precision=M.MCRT_FP64, transport_mode=mode, **run)
    ob = oracle.OracleModel(dict(cfg, run=dict(cfg["run"], seed=cfg["run"]["seed"] + 1)), mrw_gamma=2.0)
    for it in range(2):
        if it == 1:
            # the second iteration walks at the oracle's non-uniform temperatures
            # (the table's interpolation at varied T)
            g.set_temperature(o.temperature())
            ob.set_temperature(o.temperature())
        so, sg, sb = o.iterate(), g.iterate(), ob.iterate()
        print(f"iteration {it}: mrw steps {so['n_mrw']} / {sg['n_mrw']}", flush=True)
        assert so["n_mrw"] > 0
        for k in ["n_mrw", "n_cross_dust", "n_scatter", "n_absorb", "n_escape", "n_killed"]:
            assert abs(so[k] - sg[k]) <= 1e-3 * max(so[k], 1), (it, k)
        assert sg["e_escaped"] == pytest.approx(sum(s["lum"] for s in cfg["sources"]), rel=1e-12)
        eo, co = o.event_log()
        eg, cg = g.event_log()
        assert np.any(eo["type"] == oracle.EV_MRW)
        cap = eo.shape[1]
        same = co == cg
        for p in np.flatnonzero(same):
            m = min(co[p], cap)
            same[p] = all(np.array_equal(eo[f][p, :m], eg[f][p, :m]) for f in ("type", "nu", "cell"))
        print(f"  identical event sequences: {same.sum()} of {same.size}", flush=True)
        assert same.mean() >= 0.98
        ao, ag, ab = o.specific_energy(), g.specific_energy(), ob.specific_energy()
        nz = ao > 0
        assert np.array_equal(nz, ag > 0)
        # the parted packets move Adot far less than another seed does
        ratio = np.sum(np.abs(ag[nz] - ao[nz])) / np.sum(np.abs(ab[nz] - ao[nz]))
        print(f"  sum |GPU - oracle| / sum |oracle seed 2 - oracle|: {ratio:.3f}", flush=True)
        assert ratio < 0.25


def test_mrw_fp32_and_speed(M):
    # FP32 transport with the walk conserves energy and agrees with FP64 in the
    # cell temperatures; on a thick cube the walk replaces most interactions
    # (tau 30 per cell, 60 from the centre: about 2500 interactions per packet
    # without the walk)
    cfg = _thick_cube(True, n=4, tau_cell=30.0, n_packets=40000)
    plain = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT)
    walk = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, mrw_gamma=2.0)
    ref = M.Model(cfg, precision=M.MCRT_FP64, mrw_gamma=2.0)
    sp, sw, sr = plain.iterate(), walk.iterate(), ref.iterate()
    L = sum(s["lum"] for s in cfg["sources"])
    for st in (sp, sw, sr):
        assert st["e_escaped"] + st["e_killed"] == pytest.approx(L, rel=1e-9)
    assert sw["n_mrw"] > 0
    ev_plain = sp["n_scatter"] + sp["n_absorb"]
    ev_walk = sw["n_scatter"] + sw["n_absorb"] + sw["n_mrw"]
    print(f"events plain {ev_plain}, with the walk {ev_walk} ({sw['n_mrw']} steps); "
          f"transport {sp['ms_transport']:.1f} / {sw['ms_transport']:.1f} ms", flush=True)
    assert ev_walk * 2 < ev_plain
    Tw, Tr = walk.temperature(), ref.temperature()
    dust = np.asarray(cfg["rho"]).reshape(-1) > 0
    assert np.median(np.abs(Tw[dust] / Tr[dust] - 1)) < 0.01
