"""Training set, training and evaluation of the learned warm start.

The network (``mcrt.Surrogate``) maps two per-cell features of a model to
log10 T; its training targets are temperature fields that this library's own
Monte-Carlo iterations produce for a family of models.  Everything numeric
runs in the library's kernels; this module only drives them.

    python -m paper_1112_1071_amd.warmstart train --out weights.npy
    python -m paper_1112_1071_amd.warmstart evaluate --weights weights.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import synth

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart_c16.npy")

# seeds: training members, holdout members, unseen test clumps
SEED_TRAIN, SEED_HOLDOUT, SEED_TEST = 40000, 42000, 45000


# the training family: member kinds (drawn uniformly from this tuple) and the
# range of log10 of the mid-plane (disk) or radial (sphere) tau(1 um)
MEMBERS = ("sphere", "disk", "clump", "clump")
SPHERE_LOG_TAU = (-1.0, 2.0)
DISK_LOG_TAU = (-1.0, 4.3)
# the thick holdout disks the warm start is scored on: mid-plane tau(1 um) at
# least this (a cold start needs 5 or more Lucy iterations there)
THICK_DISK_TAU = 3000.0


def _family_draw(seed: int, members=MEMBERS, disk_log_tau=DISK_LOG_TAU) -> dict:
    """The random parameters of family member `seed` (kind first, so that a
    selection by kind and tau reads the same draws the member is built from)."""
    rng = np.random.default_rng(seed)
    kind = members[int(rng.integers(len(members)))]
    if kind == "clump":
        return {"kind": kind, "n_src": int(rng.integers(2, 17)), "tau": 10.0 ** rng.uniform(1.0, 2.0),
                "sigma_ln": float(rng.uniform(1.0, 2.0))}
    lo, hi = SPHERE_LOG_TAU if kind == "sphere" else disk_log_tau
    return {"kind": kind, "tau": 10.0 ** rng.uniform(lo, hi), "teff": float(rng.uniform(3000.0, 10000.0)),
            "g": float(rng.uniform(0.0, 0.8))}


def family_model(seed: int, n: int = 64, packets_per_cell: float = 10.0, n_iter: int = 10,
                 members=MEMBERS, disk_log_tau=DISK_LOG_TAU) -> dict:
    """One member of the training family at side n: a randomly parameterised
    sphere or disk (as in the batched family of uneven models) or a clump
    built with the star-forming-clump recipe at the cell size of the 128^3
    test clumps."""
    d = _family_draw(seed, members, disk_log_tau)
    kind = d["kind"]
    npk = int(packets_per_cell * n ** 3)
    if kind == "clump":
        cfg = synth.config2(n=n, n_packets=npk, n_iter=n_iter, seed=seed, gen_seed=seed,
                            n_src=d["n_src"], tau_mean=d["tau"], sigma_ln=d["sigma_ln"],
                            box=0.65 * synth.PC * n / 128)
    elif kind == "sphere":
        cfg = synth.config0(n=n, tau=d["tau"], n_packets=npk, n_iter=n_iter, seed=seed, g=d["g"],
                            teff=d["teff"])
    else:
        cfg = synth.config1(n=n, tau=d["tau"], n_packets=npk, n_iter=n_iter, seed=seed,
                            teff=d["teff"], g=d["g"], npix=1)
        cfg["observers"] = {"n_incl": 10}
    cfg["name"] = f"train{seed}-{kind}{n}"
    cfg["meta"]["family"] = kind
    return cfg


def _log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def generate(seeds, n: int = 64, packets_per_cell: float = 10.0, max_iter: int = 10, device: int = 0,
             members=MEMBERS, disk_log_tau=DISK_LOG_TAU):
    """Run the Monte-Carlo method on each member from T = 10 K until the
    convergence criterion of Sec. 2.4 (max dT/T < 1 % over the noise mask) or
    max_iter Lucy iterations, and return device tensors X [M, n^3, 3]
    (features), Y [M, n^3] (log10 T), MASK [M, n^3] (1 where the cell holds
    dust and was sampled) and the per-member iteration counts and convergence
    flags.  Member configs are built on host threads while the GPU runs."""
    import torch
    from concurrent.futures import ThreadPoolExecutor

    from . import mcrt

    M = len(seeds)
    dev = f"cuda:{device}"
    X = torch.empty((M, n ** 3, 3), dtype=torch.float32, device=dev)
    Y = torch.empty((M, n ** 3), dtype=torch.float32, device=dev)
    K = torch.empty((M, n ** 3), dtype=torch.float32, device=dev)
    iters = np.zeros(M, dtype=np.int32)
    conv = np.zeros(M, dtype=bool)
    t0 = time.time()
    pool = ThreadPoolExecutor(max_workers=8)
    futs = [pool.submit(family_model, s, n, packets_per_cell, max_iter, members, disk_log_tau)
            for s in seeds[:64]]
    for i in range(M):
        cfg = futs[i].result()
        futs[i] = None
        if i + 64 < M:
            futs.append(pool.submit(family_model, seeds[i + 64], n, packets_per_cell, max_iter, members,
                                    disk_log_tau))
        m = mcrt.Model(cfg, device=device, precision=mcrt.MCRT_FP32_TRANSPORT, stop_on_convergence=1,
                       want_noise=1, n_packets_final=1000)
        rs = m.run_all()
        iters[i], conv[i] = rs["n_iterations"], bool(rs["converged"])
        X[i] = m.features()
        T = torch.as_tensor(m.temperature(), device=dev)
        rho = torch.as_tensor(np.asarray(cfg["rho"]).reshape(-1), device=dev)
        Y[i] = torch.log10(T).float()
        K[i] = ((rho > 0) & (T > 1.0)).float()
        m.close()
        if (i + 1) % 100 == 0 or i + 1 == M:
            _log(f"# generated {i + 1}/{M} models in {time.time() - t0:.0f} s; iterations mean "
                 f"{iters[:i + 1].mean():.2f} max {iters[:i + 1].max()}, converged {conv[:i + 1].mean():.3f}")
    pool.shutdown()
    return X, Y, K, iters, conv


def train(sur, X, Y, K, epochs: int = 30, batch: int = 8, lr: float = 2e-3, holdout=None,
          seed: int = 0, log_every: int = 1):
    """Adam on the masked mean-square error of log10 T, learning rate with a
    200-step linear warm-up and a cosine decay; returns the per-epoch history."""
    import torch

    n = int(round(X.shape[1] ** (1.0 / 3.0)))
    M = X.shape[0]
    rng = np.random.default_rng(seed)
    steps = epochs * (M // batch)
    hist = []
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        perm = rng.permutation(M)
        losses = []
        for b in range(M // batch):
            idx = torch.as_tensor(perm[b * batch:(b + 1) * batch], device=X.device)
            # random axis flips: the physics is mirror-symmetric
            xb, yb, kb = X[idx], Y[idx], K[idx]
            flips = [d for d in (1, 2, 3) if rng.random() < 0.5]
            if flips:
                sh = (batch, n, n, n)
                xb = xb.reshape(*sh, 3).flip(flips).reshape(batch, -1, 3)
                yb = yb.reshape(sh).flip(flips).reshape(batch, -1)
                kb = kb.reshape(sh).flip(flips).reshape(batch, -1)
            cnt = float(kb.sum().item())
            if cnt <= 0:
                continue
            warm = min(1.0, (step + 1) / 200.0)
            cur = lr * warm * 0.5 * (1.0 + math.cos(math.pi * step / max(steps, 1)))
            losses.append(sur.train_step(xb.contiguous(), yb.contiguous(), kb.contiguous(), batch, n,
                                         lr=cur, mask_count=cnt))
            step += 1
        rec = {"epoch": ep, "train_mse": float(np.mean(losses)), "seconds": time.time() - t0}
        if holdout is not None:
            rec["holdout_mse"] = evaluate_mse(sur, *holdout)
        hist.append(rec)
        if ep % log_every == 0 or ep + 1 == epochs:
            _log("# " + json.dumps(rec))
    return hist


def evaluate_mse(sur, X, Y, K, batch: int = 8) -> float:
    n = int(round(X.shape[1] ** (1.0 / 3.0)))
    se, cnt = 0.0, 0.0
    for b in range(0, X.shape[0], batch):
        xb = X[b:b + batch].contiguous()
        nb = xb.shape[0]
        y = sur.forward(xb.reshape(-1, 3), nb, n).reshape(nb, -1)
        d = (y - Y[b:b + batch]) * K[b:b + batch]
        se += float((d * d).sum().item())
        cnt += float(K[b:b + batch].sum().item())
    return se / max(cnt, 1.0)


def test_clump(i: int, n: int = 128, n_packets: int = 250_000_000, n_iter: int = 40) -> dict:
    """Unseen clump i of the warm-start test: the star-forming-clump recipe at
    side n (same 0.65 pc box), seed SEED_TEST + i."""
    return synth.clump_config4(n=n, seed=SEED_TEST + i, n_packets=n_packets, n_iter=n_iter)


def thick_holdout_disks(count: int, n: int = 64, packets_per_cell: float = 400.0,
                        min_tau: float = THICK_DISK_TAU, n_iter: int = 40, members=MEMBERS,
                        disk_log_tau=DISK_LOG_TAU) -> list:
    """The first `count` disk members of the holdout family (seeds from
    SEED_HOLDOUT, never trained on) with mid-plane tau(1 um) >= min_tau: the
    optically thick disks where the Lucy iteration starts far from its fixed
    point."""
    out = []
    for seed in range(SEED_HOLDOUT, SEED_TEST):
        d = _family_draw(seed, members, disk_log_tau)
        if d["kind"] != "disk" or d["tau"] < min_tau:
            continue
        out.append(family_model(seed, n, packets_per_cell, n_iter, members, disk_log_tau))
        if len(out) == count:
            break
    return out


def converge(cfg: dict, sur=None, device: int = 0, **run) -> dict:
    """Lucy iterations until max dT/T < 1 % over the noise mask, from T = 10 K
    (sur None) or from the network's temperatures; wall times include the
    warm start."""
    import torch

    from . import mcrt

    m = mcrt.Model(cfg, device=device, precision=mcrt.MCRT_FP32_TRANSPORT, stop_on_convergence=1,
                   want_noise=1, n_packets_final=1000, **run)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_warm = 0.0
    if sur is not None:
        ms_warm = m.warm_start(sur)
    T0 = m.temperature() if sur is not None else np.full(m.ncell, float(cfg["run"]["t_init"]))
    rs = m.run_all()
    wall = (time.perf_counter() - t0) * 1e3
    T = m.temperature()
    rho = np.asarray(cfg["rho"]).reshape(-1)
    dust = (rho > 0) & (T > 1.0)
    e = np.abs(np.log(T0[dust] / T[dust]))
    err0 = {"median_abs_dlnT": float(np.median(e)), "p90_abs_dlnT": float(np.percentile(e, 90)),
            "mass_weighted_abs_dlnT": float(np.sum(e * rho[dust]) / np.sum(rho[dust]))}
    m.close()
    return {"iterations": rs["n_iterations"], "converged": rs["converged"],
            "first_converged": rs["first_converged"],
            "ms_to_converged": ms_warm + rs["ms_to_converged"] if rs["converged"] else None,
            "ms_warm_start": ms_warm, "wall_ms": wall, "pre_mc_error": err0,
            "max_dT": rs["last"]["max_dT"], "n_mask": rs["last"]["n_mask"]}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    t.add_argument("--n-train", type=int, default=2000)
    t.add_argument("--n-holdout", type=int, default=200)
    t.add_argument("--side", type=int, default=64)
    t.add_argument("--ppc", type=float, default=10.0)
    t.add_argument("--max-iter", type=int, default=10)
    t.add_argument("--epochs", type=int, default=25)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--lr", type=float, default=3e-4)
    t.add_argument("--clip", type=float, default=1.0)
    t.add_argument("--channels", type=int, default=16)
    t.add_argument("--members", default=",".join(MEMBERS))
    t.add_argument("--disk-log-tau", default=",".join(str(v) for v in DISK_LOG_TAU))
    t.add_argument("--history", default="")
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--n-test", type=int, default=8)
    e.add_argument("--side", type=int, default=128)
    e.add_argument("--packets", type=float, default=2.5e8)
    e.add_argument("--channels", type=int, default=16)
    args = ap.parse_args()

    from . import mcrt

    if args.cmd == "train":
        members = tuple(args.members.split(","))
        dlt = tuple(float(v) for v in args.disk_log_tau.split(","))
        X, Y, K, it_x, cv_x = generate([SEED_TRAIN + i for i in range(args.n_train)], args.side, args.ppc,
                                       args.max_iter, members=members, disk_log_tau=dlt)
        Hx, Hy, Hk, it_h, cv_h = generate([SEED_HOLDOUT + i for i in range(args.n_holdout)], args.side,
                                          args.ppc, args.max_iter, members=members, disk_log_tau=dlt)
        H = (Hx, Hy, Hk)
        sur = mcrt.Surrogate(0, args.channels, seed=1)
        sur.set_grad_clip(args.clip)
        hist = train(sur, X, Y, K, args.epochs, args.batch, args.lr, holdout=H)
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        sur.save(args.out)
        if args.history:
            with open(args.history, "w") as f:
                json.dump({"args": vars(args), "history": hist,
                           "targets": {"train_iterations": it_x.tolist(), "train_converged": cv_x.tolist(),
                                       "holdout_iterations": it_h.tolist(),
                                       "holdout_converged": cv_h.tolist()}}, f)
        print(json.dumps({"final": hist[-1]}), flush=True)
    else:
        sur = mcrt.Surrogate(0, args.channels, seed=0)
        sur.load(args.weights)
        out = []
        for i in range(args.n_test):
            cfg = test_clump(i, args.side, int(args.packets))
            cold = converge(cfg, None)
            warm = converge(cfg, sur)
            rec = {"clump": i, "cold": cold, "warm": warm}
            out.append(rec)
            print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
