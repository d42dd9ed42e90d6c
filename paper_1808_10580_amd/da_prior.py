"""Delayed-acceptance pCN with a surrogate trained on prior draws, in stages
that each fit one bounded GPU session.

Setting (the main torus problem: 168 coefficients, 49 points on a 7x7 grid,
kappa 0.01, T = 1, dt = 1e-3):
  - training pairs (u, G(u)): n_train draws u from the prior, G from the
    batched particle map (one persistent launch per 512 sets) at
    train_particles particles per point, common random numbers;
  - network 168 -> 512 -> 512 -> 512 -> 49 (GELU), BF16 matrix-core training
    with FP32 master weights (include/pm_mlp.h);
  - data y = G(u*) + N(0, gamma^2), gamma = 0.01, u* a seeded prior draw and
    G(u*) from the particle map at 1e5 particles;
  - pCN chains (Section 4.1) of n iterations each, the particle map at 1e5
    particles per point deciding acceptance (a captured graph replay with
    common random numbers); delayed acceptance screens every proposal with
    the surrogate first (stage-1 noise gamma, or gamma^2 + sigma_j^2 with
    sigma_j the surrogate's held-out error per observation: "da_aem").

Stages (each writes its results to files named on the command line; no stage
reads another's files unless given them):
    data   --part k --n-parts P --out G_k.npz    G for rows [k n/P, (k+1) n/P)
                                                 of the seeded prior draws
    train  --data G_0.npz ... --out model.npz    fit the network; G(u*), y,
                                                 and the pCN step beta from a
                                                 pilot of the plain chain
    chain  --model model.npz --kind plain|da|da_aem --iters N
           --state chain.json --trace trace.npz  run a chain to N iterations,
           [--max-seconds S]                     resuming from --state when it
                                                 exists, saving every 5,000
    report --model model.npz --trace plain=... da=...   ESS and rates (CPU)

The prior draws are regenerated from the seed in every stage, so only G
travels between stages.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

N_TRAIN = 200_000
TRAIN_PARTICLES = 20_000
CHAIN_PARTICLES = 100_000
SEED = 1808


def _setup():
    import workloads as W
    setup = W.surrogate_setup(SEED)
    wl = setup["base"]
    std = W.prior_std(wl.modes)
    return W, setup, wl, np.concatenate([std, std])


def prior_inputs(n_train: int = N_TRAIN) -> np.ndarray:
    W, _, wl, _ = _setup()
    return W.draw_prior(wl.modes, np.random.default_rng([SEED, 7]), n_train)


def _log(msg: str):
    print(f"[da-prior] {msg}", flush=True)


def stage_data(part: int, n_parts: int, out: str, n_train: int = N_TRAIN, particles: int = TRAIN_PARTICLES):
    import paper_1808_10580_amd as pm
    from paper_1808_10580_amd.surrogate import particle_dataset
    _, _, wl, _ = _setup()
    U = prior_inputs(n_train)
    lo, hi = part * n_train // n_parts, (part + 1) * n_train // n_parts
    ctx = pm.Context(0)
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    t0 = time.perf_counter()
    last = [t0]

    def progress(done, total):
        now = time.perf_counter()
        if now - last[0] > 30.0 or done == total:
            last[0] = now
            _log(f"data part {part}: {done}/{total} sets, {now - t0:.0f} s")
    G = particle_dataset(prob, wl, U[lo:hi], particles, wl.seed, progress=progress)
    sec = time.perf_counter() - t0
    np.savez(out, G=G.astype(np.float32), lo=lo, hi=hi, seconds=sec, particles=particles,
             particle_steps=float(hi - lo) * wl.n_obs * particles * wl.n_steps)
    _log(f"data part {part} done: rows {lo}..{hi}, {sec:.1f} s")
    prob.close()
    ctx.close()


def _forward(pm, ctx, wl):
    from paper_1808_10580_amd import mcmc
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    return prob, mcmc.ParticleForward(prob, wl, CHAIN_PARTICLES, wl.seed)


def stage_train(data_files, out: str, epochs: int, lr: float, lr_final: float, pilot: int = 60,
                reuse: str = None, early_stop: bool = False):
    """Fit the network; then G(u*), y and the pCN step from a pilot, or (reuse)
    take y, G(u*), gamma and beta from an earlier model file, so that chains
    started with either model sample the same posterior."""
    import paper_1808_10580_amd as pm
    from paper_1808_10580_amd import mcmc
    from paper_1808_10580_amd.surrogate import Surrogate
    _, setup, wl, prior_std = _setup()
    parts = [np.load(f) for f in data_files]
    n_train = max(int(p["hi"]) for p in parts)
    U_all = prior_inputs(n_train)
    U = np.concatenate([U_all[int(p["lo"]):int(p["hi"])] for p in parts])
    G = np.concatenate([p["G"].astype(np.float64) for p in parts])
    data_s = float(sum(float(p["seconds"]) for p in parts))
    _log(f"training on {U.shape[0]} pairs")
    ctx = pm.Context(0)
    sur = Surrogate(ctx, prior_std, wl.n_obs, seed=SEED)
    hist = sur.fit(U, G, epochs=epochs, batch=1024, lr=lr, lr_final=lr_final, early_stop=early_stop,
                   progress=lambda ep, v: _log(f"epoch {ep}: held-out rmse {v:.4f} (std units)")
                   if ep % 10 == 0 or ep == epochs - 1 or early_stop else None)
    _log(f"trained in {hist['seconds']:.1f} s, {hist['steps']} steps, kept epoch {hist.get('best_epoch', epochs - 1)}")
    prob, fwd = _forward(pm, ctx, wl)
    if reuse:
        old = np.load(reuse)
        y, g_star, gamma, beta, acc = (old["y"], old["g_star"], float(old["gamma"]), float(old["beta"]),
                                       float(old["pilot_accept"]))
    else:
        g_star = fwd(setup["u_star"])
        gamma = setup["gamma"]
        y = g_star + gamma * setup["eta"]
        # pCN step for a plain-chain acceptance rate in [0.15, 0.4] (short pilot)
        beta, acc = 0.02, 0.0
        for _ in range(6):
            pc = mcmc.start_chain(setup["u_star"], fwd, y, gamma, seed=SEED + 1)
            mcmc.pcn_steps(pc, pilot, fwd, prior_std, y, gamma, beta)
            acc = pc.n_accept / pilot
            if 0.15 <= acc <= 0.4:
                break
            beta *= 2.0 if acc > 0.4 else 0.5
    _log(f"pilot: beta {beta}, acceptance {acc:.2f}")
    val = hist["val_idx"]
    pv = sur.predict(U[val])
    st = sur.state()
    np.savez(out, **st, y=y, g_star=g_star, gamma=gamma, beta=beta, pilot_accept=acc,
             val_rmse_G=float(np.sqrt(np.mean((pv - G[val]) ** 2))),
             val_rmse_std=hist["val_rmse"][hist.get("best_epoch", epochs - 1)],
             val_rmse_hist=np.array(hist["val_rmse"]),
             err_at_ustar=float(np.sqrt(np.mean((sur(setup["u_star"]) - g_star) ** 2))),
             train_s=hist["seconds"], train_steps=hist["steps"], data_s=data_s, n_train=U.shape[0],
             epochs=epochs, lr=lr, lr_final=lr_final, best_epoch=hist.get("best_epoch", epochs - 1))
    _log(f"held-out rmse of G {float(np.sqrt(np.mean((pv - G[val]) ** 2))):.4f}; saved {out}")
    prob.close()
    ctx.close()


def stage_chain(model: str, kind: str, iters: int, state: str, trace: str, block: int = 500,
                max_seconds: float = float("inf"), save_every: int = 5000):
    """Run the chain to `iters` iterations in total (resuming from `state`
    when it exists), saving state and trace every `save_every` iterations and
    stopping early, after a save, once `max_seconds` of this session have
    passed."""
    import torch
    import paper_1808_10580_amd as pm
    from paper_1808_10580_amd import mcmc
    from paper_1808_10580_amd.surrogate import Surrogate
    _, setup, wl, prior_std = _setup()
    md = np.load(model)
    y, gamma, beta = md["y"], float(md["gamma"]), float(md["beta"])
    ctx = pm.Context(0)
    prob, fwd = _forward(pm, ctx, wl)
    sur, surf, gamma_s = None, None, None
    if kind != "plain":
        sur = Surrogate(ctx, prior_std, wl.n_obs, seed=SEED).load(md)
        surf = sur
        if kind == "da_aem":
            gamma_s = np.sqrt(gamma ** 2 + sur.err_std ** 2)
    if os.path.exists(state):
        with open(state) as fh:
            ck = json.load(fh)
        c = mcmc.Chain.resume(ck["chain"])
        seconds, calls = float(ck["seconds"]), int(ck["sessions"])
        # the trace is replaced before the state, so it holds at least c.it rows
        tr = np.load(trace)
        coords, phis = [tr["coords"][:c.it]], [tr["phi"][:c.it]]
        _log(f"{kind}: resumed at iteration {c.it}")
    else:
        c = mcmc.start_chain(setup["u_star"], fwd, y, gamma, seed=SEED + 2, surrogate=surf, gamma_s=gamma_s)
        seconds, calls = 0.0, 0
        coords, phis = [], []
    def save(chain_s):
        ck = c.checkpoint()
        ck["u"] = ck["u"].tolist()
        with open(state + ".tmp", "w") as fh:
            json.dump({"chain": ck, "seconds": chain_s, "sessions": calls + 1, "kind": kind, "beta": beta}, fh)
        np.savez(trace + ".tmp.npz", coords=np.concatenate(coords) if coords else np.zeros((0, 8)),
                 phi=np.concatenate(phis) if phis else np.zeros(0), seconds=chain_s, it=c.it,
                 n_accept=c.n_accept, n_stage1=c.n_stage1, n_forward=c.n_forward)
        os.replace(trace + ".tmp.npz", trace)
        os.replace(state + ".tmp", state)
        _log(f"{kind}: saved at iteration {c.it}, {chain_s:.0f} s of chain time")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start_it = c.it
    while c.it < iters:
        nb = min(block, iters - c.it)
        if kind == "plain":
            mcmc.pcn_steps(c, nb, fwd, prior_std, y, gamma, beta)
        else:
            mcmc.da_pcn_steps(c, nb, fwd, surf, prior_std, y, gamma, beta, gamma_s=gamma_s)
        S = np.array(c.samples)
        coords.append(S[:, :8].copy())
        phis.append(np.array(c.phis))
        c.samples.clear()
        c.phis.clear()
        el = time.perf_counter() - t0
        if c.it % 2500 == 0 or c.it == iters:
            done = c.it - start_it
            _log(f"{kind}: iteration {c.it} ({done} this session, {el:.0f} s, {done / el:.1f}/s, "
                 f"accepted {c.n_accept}, particle maps {c.n_forward})")
        if c.it % save_every == 0 or c.it == iters or el > max_seconds:
            torch.cuda.synchronize()
            save(seconds + time.perf_counter() - t0)
            if el > max_seconds:
                break
    prob.close()
    ctx.close()


def report(model: str, traces: dict) -> dict:
    """Samples/s and the effective sample size (Geyer) of the first 8
    coefficients and of the misfit, per chain; ratios against the plain chain."""
    from paper_1808_10580_amd import mcmc
    md = np.load(model)
    out = {"n_train": int(md["n_train"]), "train_s": float(md["train_s"]), "data_s": float(md["data_s"]),
           "val_rmse_G": float(md["val_rmse_G"]),
           "val_rmse_std": float(np.min(md["val_rmse_hist"])) if "best_epoch" in md else float(md["val_rmse_std"]),
           "err_at_ustar": float(md["err_at_ustar"]), "gamma": float(md["gamma"]), "beta": float(md["beta"]),
           "surrogate_err_std_mean": float(np.mean(md["err_std"]))}
    for kind, path in traces.items():
        tr = np.load(path)
        it, sec = int(tr["it"]), float(tr["seconds"])
        e = min(mcmc.ess(tr["coords"][:, c]) for c in range(8))
        e_phi = mcmc.ess(tr["phi"])
        out[kind] = {"iterations": it, "seconds": sec, "samples_per_s": it / sec, "accept_rate": int(tr["n_accept"]) / it,
                     "stage1_pass_rate": int(tr["n_stage1"]) / it, "particle_map_calls": int(tr["n_forward"]),
                     "ess_min_first8": e, "ess_phi": e_phi, "ess_per_s": e / sec, "ess_phi_per_s": e_phi / sec}
    if "plain" in out:
        for kind in traces:
            if kind != "plain":
                out[f"{kind}_vs_plain"] = {
                    "samples_per_s": out[kind]["samples_per_s"] / out["plain"]["samples_per_s"],
                    "ess_per_s": out[kind]["ess_per_s"] / max(out["plain"]["ess_per_s"], 1e-300),
                    "ess_phi_per_s": out[kind]["ess_phi_per_s"] / max(out["plain"]["ess_phi_per_s"], 1e-300)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("stage", choices=["data", "train", "chain", "report"])
    ap.add_argument("--part", type=int, default=0)
    ap.add_argument("--n-parts", type=int, default=1)
    ap.add_argument("--n-train", type=int, default=N_TRAIN)
    ap.add_argument("--particles", type=int, default=TRAIN_PARTICLES)
    ap.add_argument("--out", default=None)
    ap.add_argument("--data", nargs="*", default=[])
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=5e-5)
    ap.add_argument("--model", default=None)
    ap.add_argument("--reuse", default=None, help="train: take y, G(u*), gamma, beta from this model file")
    ap.add_argument("--early-stop", action="store_true", help="train: keep the epoch with the lowest held-out error")
    ap.add_argument("--kind", default="plain", choices=["plain", "da", "da_aem"])
    ap.add_argument("--iters", type=int, default=1000)
    ap.add_argument("--state", default=None)
    ap.add_argument("--trace", nargs="*", default=[])
    ap.add_argument("--max-seconds", type=float, default=float("inf"))
    a = ap.parse_args()
    if a.stage == "data":
        stage_data(a.part, a.n_parts, a.out, a.n_train, a.particles)
    elif a.stage == "train":
        stage_train(a.data, a.out, a.epochs, a.lr, a.lr_final, reuse=a.reuse, early_stop=a.early_stop)
    elif a.stage == "chain":
        stage_chain(a.model, a.kind, a.iters, a.state, a.trace[0], max_seconds=a.max_seconds)
    else:
        print(json.dumps(report(a.model, dict(t.split("=", 1) for t in a.trace))))
    return 0


if __name__ == "__main__":
    sys.exit(main())
