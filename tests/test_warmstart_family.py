"""Host-side checks of the warm-start workloads: the thick holdout disks are
disk members of the holdout seed range (never trained on) with mid-plane
tau(1 um) >= the threshold, and the family draw that selects them is the one
family_model makes."""
from paper_1112_1071_amd import warmstart


def test_thick_holdout_disks():
    cfgs = warmstart.thick_holdout_disks(3, n=16, packets_per_cell=2.0)
    assert len(cfgs) == 3
    seeds = []
    for c in cfgs:
        assert c["meta"]["family"] == "disk"
        assert c["meta"]["tau_1um"] >= 100.0
        seed = int(c["name"].split("-")[0].replace("train", ""))
        assert warmstart.SEED_HOLDOUT <= seed < warmstart.SEED_HOLDOUT + 100000
        assert seed < warmstart.SEED_TEST
        seeds.append(seed)
        assert c["run"]["n_packets"] == 2 * 16 ** 3
    assert seeds == sorted(seeds) and len(set(seeds)) == 3
    # the same members, built directly
    for s, c in zip(seeds, cfgs):
        d = warmstart.family_model(s, 16, 2.0, 40)
        assert d["meta"]["family"] == "disk" and d["meta"]["tau_1um"] == c["meta"]["tau_1um"]


def test_thick_disk_threshold():
    thin = warmstart.thick_holdout_disks(2, n=16, packets_per_cell=1.0, min_tau=1e-3)
    thick = warmstart.thick_holdout_disks(2, n=16, packets_per_cell=1.0, min_tau=500.0)
    assert all(c["meta"]["tau_1um"] >= 500.0 for c in thick)
    assert thin[0]["name"] != thick[0]["name"]


def test_committed_network_was_trained_on_this_family():
    # the committed weights' training run used the family and target settings
    # the module builds by default, so the holdout disks the warm start is
    # scored on are members of the holdout family the network never saw
    import json
    import os

    h = json.load(open(os.path.join(os.path.dirname(warmstart.__file__), "weights",
                                    "warmstart_c16_history.json")))
    a = h["args"]
    assert tuple(a["members"].split(",")) == warmstart.MEMBERS
    assert tuple(float(v) for v in a["disk_log_tau"].split(",")) == warmstart.DISK_LOG_TAU
    assert a["n_train"] == 2000 and a["n_holdout"] == 200 and a["side"] == 64
    # targets: every member iterated to the convergence criterion
    t = h["targets"]
    assert len(t["train_iterations"]) == 2000 and all(t["train_converged"])
    assert all(t["holdout_converged"])
    # the thick holdout disks come from the holdout seed range
    for c in warmstart.thick_holdout_disks(2, n=16, packets_per_cell=1.0):
        seed = int(c["name"].split("-")[0].replace("train", ""))
        assert warmstart.SEED_HOLDOUT <= seed < warmstart.SEED_TEST
        assert c["meta"]["tau_1um"] >= warmstart.THICK_DISK_TAU
