"""GPU (HIP, gfx950) vs the FP64 CPU oracle, through the C ABI.

Same-stream parity (FP64 transport, same seed): identical packet event
sequences, absorption tallies and temperatures equal to summation-order
rounding, identical counters and SED/image counts.  FP32 transport and
independent seeds: statistical agreement (z-tests against Monte-Carlo
error).  Tolerances:
  * Adot relative 1e-9 (FP64 atomics reorder the sums; each cell sums O(1e3)
    terms of one sign, so the rounding stays near 1e-13);
  * T relative 1e-8 (the GPU inverts a cubic Hermite table of ln Adot(ln T)
    whose interpolation error is below 1e-10; the oracle solves Eq. 3 to 1e-13);
  * per-cell T within 1 % where the oracle's sigma_T/T < 0.3 % (FP32, other seeds);
  * SED bins |z| < 4 in >= 99.9 % of bins.
"""
import math

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


def compare_logs(eo, co, eg, cg):
    assert np.array_equal(co, cg), f"event counts differ for {np.sum(co != cg)} packets"
    cap = eo.shape[1]
    idx = np.arange(cap)[None, :] < np.minimum(co, cap)[:, None]
    for f in ["packet", "index", "type", "nu", "incl"]:
        a, b = eo[f][idx], eg[f][idx]
        assert np.array_equal(a, b), f"field {f} differs at {np.sum(a != b)} events"
    assert np.array_equal(eo["cell"][idx], eg["cell"][idx])


def test_event_sequences_optically_thin(M):
    # config 0 at tau(1 um) = 0.1: packets 0..9999 of iteration 0, GPU FP64 vs oracle
    cfg = synth.config0(tau=0.1, n_packets=100000, n_iter=1)
    run = dict(event_log_packets=10000, event_log_cap=64)
    o = oracle.OracleModel(cfg, **run)
    g = M.Model(cfg, precision=M.MCRT_FP64, **run)
    so, sg = o.iterate(), g.iterate()
    eo, co = o.event_log()
    eg, cg = g.event_log()
    assert (co > 2).mean() > 0.05  # a good fraction of packets interact
    compare_logs(eo, co, eg, cg)
    for k in ["n_cross_dust", "n_cross_empty", "n_scatter", "n_absorb", "n_escape", "n_killed"]:
        assert so[k] == sg[k], k


@pytest.fixture(scope="module")
def same_stream_runs(M):
    cfg = synth.config0(n_packets=100000, n_iter=3, images=True)
    run = dict(want_noise=1, bin_every_iteration=1)
    o = oracle.OracleModel(cfg, **run)
    g = M.Model(cfg, precision=M.MCRT_FP64, **run)
    out = []
    for _ in range(3):
        so, sg = o.iterate(), g.iterate()
        ao, sigo = o.specific_energy(with_sigma=True)
        ag, sigg = g.specific_energy(with_sigma=True)
        out.append((so, sg, ao, ag, sigo, sigg, o.temperature(), g.temperature(), o.sed(), g.sed(),
                    o.images(), g.images()))
    return cfg, out


def test_same_stream_adot_and_temperature(same_stream_runs):
    cfg, out = same_stream_runs
    for so, sg, ao, ag, sigo, sigg, To, Tg, *_ in out:
        for k in ["n_cross_dust", "n_cross_empty", "n_scatter", "n_absorb", "n_escape",
                  "n_unsampled", "n_r", "n_mask"]:
            assert so[k] == sg[k], k
        assert np.array_equal(ao > 0, ag > 0)
        nz = ao > 0
        assert np.max(np.abs(ag[nz] / ao[nz] - 1)) < 1e-9
        assert np.max(np.abs(sigg[nz] / sigo[nz] - 1)) < 1e-9
        assert np.max(np.abs(Tg / To - 1)) < 1e-8
        assert sg["e_escaped"] == pytest.approx(so["e_escaped"], rel=1e-12)
        for k in ["q", "delta", "max_dT", "p999_dT"]:
            if math.isfinite(so[k]):
                assert sg[k] == pytest.approx(so[k], rel=1e-7), k
            else:
                assert not math.isfinite(sg[k]), k


def test_same_stream_sed_and_images(same_stream_runs):
    cfg, out = same_stream_runs
    so, sg, *_, sedo, sedg, imo, img = out[-1]
    assert np.array_equal(sedo[2], sedg[2])
    assert np.allclose(sedg[0], sedo[0], rtol=1e-12, atol=0)
    assert np.allclose(sedg[1], sedo[1], rtol=1e-12, atol=0)
    assert imo[0].sum() > 0
    # direct light of the central star projects exactly onto the image centre,
    # a corner shared by four pixels: which of them receives it is decided by
    # rounding, so compare the 2x2 central block as one and every other pixel
    for a, b in [(img[0], imo[0]), (img[1], imo[1])]:
        c = a.shape[-1] // 2
        ca = a[..., c - 1:c + 1, c - 1:c + 1].sum(axis=(-1, -2))
        cb = b[..., c - 1:c + 1, c - 1:c + 1].sum(axis=(-1, -2))
        assert np.allclose(ca, cb, rtol=1e-12, atol=0)
        a, b = a.copy(), b.copy()
        a[..., c - 1:c + 1, c - 1:c + 1] = 0
        b[..., c - 1:c + 1, c - 1:c + 1] = 0
        assert np.allclose(a, b, rtol=1e-12, atol=0)


def test_final_pass_same_stream(M):
    cfg = synth.config0(n=16, n_packets=50000, n_iter=2, n_bins=50, images=True)
    o = oracle.OracleModel(cfg)
    g = M.Model(cfg, precision=M.MCRT_FP64)
    for _ in range(2):
        o.iterate()
        g.iterate()
    so, sg = o.final_pass(), g.final_pass()
    assert so["n_escape"] == sg["n_escape"]
    assert np.array_equal(o.sed()[2], g.sed()[2])
    assert np.allclose(g.sed()[0], o.sed()[0], rtol=1e-12, atol=0)


def sed_z(sa, s2a, sb, s2b, eps):
    var = s2a + s2b
    floor = (eps ** 2) * ((sa == 0) ^ (sb == 0))
    var = np.maximum(var, floor)
    both0 = (sa == 0) & (sb == 0)
    z = np.zeros_like(sa)
    ok = ~both0
    z[ok] = (sa[ok] - sb[ok]) / np.sqrt(var[ok])
    return z


@pytest.mark.parametrize("precision", [0, 1])
def test_independent_seed_statistics(M, precision):
    # oracle and GPU with different seeds agree within Monte-Carlo error
    cfg = synth.config0(n_packets=200000, n_iter=3)
    o = oracle.OracleModel(cfg, want_noise=1, seed=11)
    g = M.Model(cfg, precision=precision, want_noise=1, seed=12)
    for _ in range(3):
        o.iterate()
        g.iterate()
    To, Tg = o.temperature(), g.temperature()
    ao, so_ = o.specific_energy(with_sigma=True)
    ag, sg_ = g.specific_energy(with_sigma=True)
    rho = cfg["rho"].ravel()
    m = (rho > 0) & (ao > 0) & (ag > 0)
    za = (ag[m] - ao[m]) / np.sqrt(so_[m] ** 2 + sg_[m] ** 2)
    assert np.mean(np.abs(za) < 4) >= 0.999 - 3 / m.sum() ** 0.5
    assert abs(np.mean(za)) < 0.1
    o.final_pass()
    g.final_pass()
    so, s2o, _ = o.sed()
    sg, s2g, _ = g.sed()
    eps = cfg["sources"][0]["lum"] / cfg["run"]["n_packets"]
    z = sed_z(so, s2o, sg, s2g, eps)
    assert np.mean(np.abs(z) < 4) >= 0.999 - 1e-9 or np.sum(np.abs(z) >= 4) <= 1


def test_fp32_same_seed_error_report(M):
    # FP32 transport from the same random stream as the FP64 oracle: per-result
    # errors; enough packets that many cells reach sigma_T/T < 0.3 %
    cfg = synth.config0(n_packets=8_000_000, n_iter=2)
    o = oracle.OracleModel(cfg, want_noise=1, event_log_packets=10000, event_log_cap=64)
    g = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, want_noise=1, event_log_packets=10000,
                event_log_cap=64)
    for i in range(2):
        o.iterate()
        g.iterate()
        if i == 0:
            eo, co = o.event_log()
            eg, cg = g.event_log()
            same = np.array([co[p] == cg[p] and np.array_equal(eo[p, : min(co[p], 64)]["type"],
                                                                 eg[p, : min(cg[p], 64)]["type"])
                             for p in range(len(co))])
            # FP32 uniforms keep 24 of the 52 bits: a few per cent of packets diverge
            assert same.mean() > 0.9
    To, Tg = o.temperature(), g.temperature()
    a, s = o.specific_energy(with_sigma=True)
    ag = g.specific_energy()
    rho = cfg["rho"].ravel()
    slope_m = (rho > 0) & (a > 0)
    sig_T = (s[slope_m] / a[slope_m]) / 4.5
    quiet = sig_T < 0.003
    rel = np.abs(Tg[slope_m][quiet] / To[slope_m][quiet] - 1)
    assert quiet.sum() > 1000
    assert np.all(rel < 0.01), rel.max()
    # the final pass at these temperatures: SED bins
    o.final_pass()
    g.final_pass()
    so, s2o, no = o.sed()
    sg, _, ng = g.sed()
    # a bin's sum over a random number of packets: variance sum of squares
    full = no > 100
    z = np.abs(sg[full] - so[full]) / np.sqrt(2.0 * s2o[full])
    assert np.mean(z < 4) >= 0.999
    za = np.abs(ag[slope_m] - a[slope_m]) / s[slope_m]
    print(f"FP32 transport against the FP64 oracle, same stream: identical event sequences "
          f"{same.mean():.4f} of {len(same)} packets; T in cells with sigma_T/T < 0.3 %: median "
          f"{np.median(rel):.2e}, max {rel.max():.2e} ({quiet.sum()} cells); Adot |diff|/sigma: "
          f"median {np.median(za):.2f}, p99.9 {np.quantile(za, 0.999):.2f}; SED bins with > 100 "
          f"packets: |z| < 4 in {np.mean(z < 4):.4f} of {full.sum()}, median relative difference "
          f"{np.median(np.abs(sg[full] / so[full] - 1)):.2e}", flush=True)


def test_edge_cases_same_stream(M):
    # empty grid, a single cell, a ragged non-cubic grid with an off-centre
    # source, a packet count that is not a multiple of the block, and kills
    base = synth.config0(n=8, n_packets=12345, n_iter=1, n_bins=20)
    cases = []
    c = dict(base)
    c["rho"] = np.zeros_like(base["rho"])
    cases.append(("empty", c, {}))
    c = dict(base)
    c["grid"] = {"n": [1, 1, 1], "lo": [-1.0, -1.0, -1.0], "hi": [1.0, 1.0, 1.0]}
    c["rho"] = np.array([0.4])
    c["sources"] = [{"pos": [0.0, 0.0, 0.0], "lum": 1.0, "teff": 3000.0}]
    cases.append(("one-cell", c, {}))
    c = dict(base)
    rng = np.random.default_rng(5)
    c["grid"] = {"n": [7, 5, 3], "lo": [-3e13, -1e13, 0.0], "hi": [4e13, 2e13, 1.5e13]}
    c["rho"] = rng.uniform(0, 2e-15, size=(3, 5, 7)) * (rng.random((3, 5, 7)) > 0.3)
    c["sources"] = [{"pos": [1.1e13, 0.3e13, 0.7e13], "lum": synth.L_SUN, "teff": 8000.0},
                    {"pos": [-3e13, -1e13, 0.0], "lum": 0.5 * synth.L_SUN, "teff": 3000.0}]
    cases.append(("ragged", c, {}))
    cases.append(("equal-sampling", c, {"source_sampling": 1}))
    c2 = dict(base)
    c2["rho"] = base["rho"] * 20
    cases.append(("kills", c2, {"max_events": 3}))
    for name, cfg, extra in cases:
        run = dict(event_log_packets=2000, event_log_cap=16, **extra)
        o = oracle.OracleModel(cfg, **run)
        g = M.Model(cfg, precision=M.MCRT_FP64, **run)
        so, sg = o.iterate(), g.iterate()
        for k in ["n_cross_dust", "n_cross_empty", "n_scatter", "n_absorb", "n_escape", "n_killed"]:
            assert so[k] == sg[k], (name, k)
        L = sum(s["lum"] for s in cfg["sources"])
        assert sg["e_escaped"] + sg["e_killed"] == pytest.approx(L, rel=1e-12), name
        eo, co = o.event_log()
        eg, cg = g.event_log()
        compare_logs(eo, co, eg, cg)
        ao, ag = o.specific_energy(), g.specific_energy()
        nz = ao > 0
        assert np.array_equal(nz, ag > 0), name
        if nz.any():
            assert np.max(np.abs(ag[nz] / ao[nz] - 1)) < 1e-9, name
        assert np.max(np.abs(g.temperature() / o.temperature() - 1)) < 1e-8, name


def test_abi_errors(M):
    cfg = synth.config0(n=4, n_packets=100, n_bins=10)
    g = M.Model(cfg)
    L, h = g.L, g.h
    import ctypes as C

    lo = np.zeros(3)
    hi = np.ones(3)
    assert L.mcrt_set_grid(h, 0, 1, 1, lo.ctypes.data, hi.ctypes.data) == -1
    bad = np.array([1.0, -1.0])
    g2 = M.Model(cfg)
    assert g2.L.mcrt_set_density(g2.h, bad.ctypes.data, 2) == -6  # size mismatch
    rho = np.full(64, -1.0)
    assert g2.L.mcrt_set_density(g2.h, rho.ctypes.data, 64) == -1
    rho = np.full(64, np.nan)
    assert g2.L.mcrt_set_density(g2.h, rho.ctypes.data, 64) == -1
    T = np.zeros(64)
    assert g2.L.mcrt_set_temperature(g2.h, T.ctypes.data, 64) == -1
    out = np.zeros(10)
    assert g2.L.mcrt_get_temperature(g2.h, out.ctypes.data, 10) in (-6, -2)
    # iterate before setup on a fresh model
    h3 = C.c_void_p()
    assert L.mcrt_create(C.byref(h3), 0) == 0
    st = M.IterStats()
    assert L.mcrt_iterate(h3, C.byref(st)) == -2
    L.mcrt_destroy(h3)
    L.mcrt_destroy(None)
    # groups above 256 threads exist for the FP32 tiled sweeps only, up to 768
    for bad_run in (dict(precision=M.MCRT_FP64, transport_mode=1, block_size=512),
                    dict(precision=M.MCRT_FP32_TRANSPORT, transport_mode=0, block_size=512),
                    dict(precision=M.MCRT_FP32_TRANSPORT, transport_mode=1, block_size=832),
                    dict(precision=M.MCRT_FP32_TRANSPORT, transport_mode=1, block_size=96)):
        with pytest.raises(M.MCRTError):
            M.Model(cfg, **bad_run)


@pytest.mark.parametrize("variant", [
    # per-lane persistent walk (transport_mode 0)
    dict(transport_mode=0, walk_batch=1, grid_layout=0, tally_copies=1),
    dict(transport_mode=0, walk_batch=2, grid_layout=1, tally_copies=8),
    dict(transport_mode=0, walk_batch=4, grid_layout=1, tally_copies=1, block_size=128),
    dict(transport_mode=0, walk_batch=8, grid_layout=0, tally_copies=8, defer_lanes=1),
    dict(transport_mode=0, walk_batch=8, grid_layout=1, tally_copies=8, defer_lanes=64, block_size=64),
    # tiled sweeps: tiles of 16x16x{4,8} (ragged at the grid edges), yields
    # after every interaction (visit_events=1), lone-lane event handling
    dict(transport_mode=1, tile_z=8, walk_batch=4),
    dict(transport_mode=1, tile_z=4, walk_batch=1, visit_events=1),
    dict(transport_mode=1, tile_z=8, walk_batch=2, defer_lanes=1, visit_events=3),
    dict(transport_mode=1, tile_xy=32, tile_z=8, walk_batch=4),
    dict(transport_mode=1),  # the defaults: 16x16x32 tiles, full-wave deferral
])
def test_launch_variants_same_stream(M, variant):
    # every launch configuration the library offers gives the oracle's packets
    cfg = synth.config0(n=20, tau=2.0, n_packets=30000, n_iter=1, n_bins=40)
    cfg["grid"]["n"] = [20, 18, 13]  # ragged bricks on every axis
    cfg["rho"] = np.resize(cfg["rho"], (13, 18, 20))
    run = dict(event_log_packets=3000, event_log_cap=32)
    o = oracle.OracleModel(cfg, **run)
    g = M.Model(cfg, precision=M.MCRT_FP64, **run, **variant)
    so, sg = o.iterate(), g.iterate()
    for k in ["n_cross_dust", "n_cross_empty", "n_scatter", "n_absorb", "n_escape"]:
        assert so[k] == sg[k], k
    eo, co = o.event_log()
    eg, cg = g.event_log()
    compare_logs(eo, co, eg, cg)
    ao, ag = o.specific_energy(), g.specific_energy()
    nz = ao > 0
    assert np.array_equal(nz, ag > 0)
    assert np.max(np.abs(ag[nz] / ao[nz] - 1)) < 1e-9


@pytest.mark.parametrize("tiles", [dict(tile_xy=16, tile_z=4, block_size=256),
                                   dict(tile_xy=16, tile_z=32, block_size=256),
                                   dict(tile_xy=32, tile_z=4, block_size=128),
                                   # the FP32 default: one 8-wave group per 32x32x16
                                   # tile (128 KB of LDS; 32x32x8 with Sum w^2 kept)
                                   dict()])
def test_tiled_fp32_equals_persistent_fp32(M, tiles):
    # FP32 transport: both modes follow identical packet histories in the first
    # iteration (same counters exactly) and add the same FP32 products w l kappa
    # into FP64 sums (the tiled mode in LDS, flushed to the FP64 tally), so
    # Adot and its noise estimate agree to FP64 summation order (1e-9).  The
    # second iteration re-emits from temperatures that differ at that level,
    # which could flip a rare emission-row choice; a flipped packet takes
    # another path from there on, moving the cells it crosses by about one
    # packet's contribution, within their Monte-Carlo error: counters agree to
    # 1e-4, Adot to 1e-4 in 99 % of the cells and within 3 sigma in 99.9 %.
    cfg = synth.config2(n=48, n_packets=400000, n_iter=2, gen_seed=45777, n_src=12,
                        box=0.65 * synth.PC * 48 / 128)
    a = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, want_noise=1, transport_mode=0)
    b = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, want_noise=1, transport_mode=1, **tiles)
    for it in range(2):
        sa, sb = a.iterate(), b.iterate()
        for k in ["n_cross_dust", "n_cross_empty", "n_scatter", "n_absorb", "n_escape", "n_killed"]:
            if it == 0:
                assert sa[k] == sb[k], (it, k)
            else:
                assert abs(sa[k] - sb[k]) <= 1e-4 * max(sa[k], 1), (it, k)
        assert sb["n_sweeps"] > 0
        aa, sga = a.specific_energy(with_sigma=True)
        ab, sgb = b.specific_energy(with_sigma=True)
        nz = (aa > 0) & (ab > 0)
        rel = np.abs(ab[nz] / aa[nz] - 1)
        srel = np.abs(sgb[nz] - sga[nz]) / sga[nz]
        if it == 0:
            assert np.array_equal(aa > 0, ab > 0)
            assert rel.max() < 1e-9 and srel.max() < 1e-9, it
            np.testing.assert_allclose(b.temperature(), a.temperature(), rtol=1e-9)
        else:
            z = np.abs(ab[nz] - aa[nz]) / np.sqrt(sga[nz] ** 2 + sgb[nz] ** 2)
            print(f"iteration {it}: rel q99 {np.quantile(rel, 0.99):.2e} q999 {np.quantile(rel, 0.999):.2e} "
                  f"max {rel.max():.2e}; z>3 in {np.mean(z > 3):.2e} of cells, max z {z.max():.2f}")
            assert np.quantile(rel, 0.99) < 1e-4, it
            assert np.mean(z < 3) > 0.999, it


@pytest.mark.parametrize("mode", [0, 1])
def test_peeloff_same_stream(M, mode):
    # peeling-off (Sec. 2.6.2) in the final pass: the same events peel the same
    # weights toward each observer as in the oracle (FP64, same seed)
    cfg = synth.config0(n=24, tau=1.0, n_packets=40000, n_iter=1, n_bins=40, images=True)
    cfg["peeloff"] = {"dirs": [[0.0, 0.0, 1.0], [0.6, 0.0, 0.8], [0.48, -0.6, 0.64]]}
    o = oracle.OracleModel(cfg)
    g = M.Model(cfg, precision=M.MCRT_FP64, transport_mode=mode)
    o.iterate(), g.iterate()
    o.final_pass(), g.final_pass()
    so, so2 = o.peeled_sed()
    sg, sg2 = g.peeled_sed()
    assert so.shape == (3, 2, 40) and np.all(so[:, 0].sum(axis=1) > 0) and np.all(so[:, 1].sum(axis=1) > 0)
    nz = so != 0
    assert np.array_equal(nz, sg != 0)
    np.testing.assert_allclose(sg[nz], so[nz], rtol=1e-9)
    np.testing.assert_allclose(sg2[nz], so2[nz], rtol=1e-9)
    io, _ = o.peeled_images()
    ig, _ = g.peeled_images()
    np.testing.assert_allclose(ig.sum(axis=(2, 3)), io.sum(axis=(2, 3)), rtol=1e-9)
    # a point projected exactly onto a pixel edge may land on either side
    close = np.isclose(ig, io, rtol=1e-9, atol=0)
    assert close.mean() > 0.999


@pytest.mark.parametrize("sampling", [0, 1])
def test_sources_on_tile_walls_same_stream(M, sampling):
    # Sources exactly on cell walls that are also tile walls (FP64 tiles are
    # 16 cells wide): a packet whose direction points to the lower side starts
    # in the lower cell (Sec. 2.2 emission; reading of a position on a wall),
    # which lies in the neighbouring tile.  The tiled emission registers every
    # packet with the tile of that cell, so the FP64 tiled pass equals the
    # oracle's event by event, and the FP32 tiled pass equals the FP32 per-lane
    # walk.  Cell size 2^43 cm keeps every wall position exact.
    base = synth.config0(n=32, n_packets=20000, n_iter=1, n_bins=20)
    dx = 2.0 ** 43
    cfg = dict(base)
    cfg["grid"] = {"n": [32, 32, 32], "lo": [0.0, 0.0, 0.0], "hi": [32 * dx] * 3}
    cfg["sources"] = [{"pos": [16 * dx, 16 * dx, 16.5 * dx], "lum": synth.L_SUN, "teff": 6000.0},
                      {"pos": [8 * dx, 16 * dx, 16 * dx], "lum": 0.5 * synth.L_SUN, "teff": 4000.0},
                      {"pos": [0.0, 20.25 * dx, 32 * dx - dx / 4], "lum": 0.25 * synth.L_SUN, "teff": 3000.0}]
    run = dict(event_log_packets=2000, event_log_cap=16, source_sampling=sampling)
    o = oracle.OracleModel(cfg, **run)
    g = M.Model(cfg, precision=M.MCRT_FP64, **run)
    assert g.run["transport_mode"] == 1
    so, sg = o.iterate(), g.iterate()
    for k in ["n_cross_dust", "n_cross_empty", "n_scatter", "n_absorb", "n_escape", "n_killed"]:
        assert so[k] == sg[k], k
    assert sg["n_escape"] + sg["n_killed"] == 20000
    eo, co = o.event_log()
    eg, cg = g.event_log()
    compare_logs(eo, co, eg, cg)
    ao, ag = o.specific_energy(), g.specific_energy()
    o.close()
    g.close()
    nz = ao > 0
    assert np.array_equal(nz, ag > 0)
    assert np.max(np.abs(ag[nz] / ao[nz] - 1)) < 1e-9
    a = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, transport_mode=0, source_sampling=sampling)
    b = M.Model(cfg, precision=M.MCRT_FP32_TRANSPORT, transport_mode=1, source_sampling=sampling)
    sa, sb = a.iterate(), b.iterate()
    for k in ["n_cross_dust", "n_cross_empty", "n_scatter", "n_absorb", "n_escape", "n_killed"]:
        assert sa[k] == sb[k], k
    aa, ab = a.specific_energy(), b.specific_energy()
    a.close()
    b.close()
    nz = aa > 0
    assert np.array_equal(nz, ab > 0)
    assert np.max(np.abs(ab[nz] / aa[nz] - 1)) < 1e-9
