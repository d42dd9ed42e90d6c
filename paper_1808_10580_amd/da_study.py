"""Plain pCN vs delayed-acceptance pCN with the learned surrogate.

    python -m paper_1808_10580_amd.da_study [--n-train 8192] [--train-particles 10000] [--iters 2000]
                                            [--horizon T] [--engine auto|valu]

Setting (the surrogate workload): the main torus problem (168 coefficients,
49 observation points, T = 1), synthetic data y = G(u*) + N(0, gamma^2),
gamma = 0.01, with u* a prior draw and G(u*) from the particle map at 1e5
particles.  Both chains evaluate the particle map with 1e5 particles per point
(a captured graph replay, common random numbers) to decide acceptance; the
delayed-acceptance chain screens proposals with the surrogate first.  Both
start at u* (no burn-in) and use the same pCN step beta, chosen by a short
pilot of the plain chain for an acceptance rate between 0.15 and 0.4.

The posterior is far narrower than the prior, so a network fitted to prior
draws only learns the prior mean of G; the training inputs are pCN moves of
size 2 beta around the pilot chain's states (where the chains live), their
outputs the batched particle map at a reduced particle count.

--horizon sets the observation time (default the workload's T = 1, where the
flow has mixed the particles far apart); shorter horizons give a smoother,
less chaotic G.  --engine selects the FP32 velocity engine of the particle map.

Three chains: plain pCN, delayed acceptance with the surrogate misfit at the
data noise gamma, and delayed acceptance with an approximation-error model
(stage-1 noise gamma^2 + sigma_j^2, sigma_j the surrogate's held-out error per
observation).  Output: one JSON line with samples/s, particle-map calls,
acceptance rates and the effective sample size (Geyer) of the misfit trace and
of the first 8 coefficients for every chain, plus the surrogate's training
time and held-out error.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import time

import numpy as np


def run(n_train=8192, train_particles=10_000, iters=2000, pilot=60, chain_particles=100_000, seed=1808,
        epochs=200, verbose=True, dump=None, dataset_only=False, horizon=None, engine="auto"):
    import torch

    import paper_1808_10580_amd as pm
    import workloads as W
    from paper_1808_10580_amd import mcmc
    from paper_1808_10580_amd.surrogate import Surrogate, particle_dataset

    setup = W.surrogate_setup(seed)
    wl = setup["base"]
    if horizon is not None:
        wl = dataclasses.replace(wl, T=float(horizon))
    gamma = setup["gamma"]
    std = W.prior_std(wl.modes)
    prior_std = np.concatenate([std, std])
    ctx = pm.Context(0)
    ctx.set_velocity_engine(engine)
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    if engine == "valu":
        prob.autotune_time(wl.u, wl.obs, wl.kappa, wl.dt, chain_particles, wl.seed, n_probe_steps=50)
    out = {"n_train": n_train, "train_particles": train_particles, "chain_particles": chain_particles,
           "iters": iters, "gamma": gamma, "horizon": wl.T, "engine": engine}

    # data y = G(u*) + gamma eta
    fwd = mcmc.ParticleForward(prob, wl, chain_particles, wl.seed)
    g_star = fwd(setup["u_star"])
    y = g_star + gamma * setup["eta"]

    # pilot: choose beta for plain-pCN acceptance in [0.15, 0.4]
    beta = 0.02
    for _ in range(6):
        pc = mcmc.start_chain(setup["u_star"], fwd, y, gamma, seed=seed + 1)
        mcmc.pcn_steps(pc, pilot, fwd, prior_std, y, gamma, beta)
        acc = pc.n_accept / pilot
        if 0.15 <= acc <= 0.4:
            break
        beta *= 2.0 if acc > 0.4 else 0.5
    out["beta"] = beta
    out["pilot_accept"] = acc

    # training pairs: pCN moves of size 2 beta around the pilot chain's states,
    # evaluated by the batched particle map
    rng = np.random.default_rng([seed, 6])
    centres = np.array(pc.samples)[rng.integers(0, len(pc.samples), n_train)]
    bt = min(2.0 * beta, 1.0)
    U = math.sqrt(1.0 - bt * bt) * centres + bt * W.draw_prior(wl.modes, rng, n_train)
    t0 = time.perf_counter()
    G = particle_dataset(prob, wl, U, train_particles, wl.seed)
    out["dataset_s"] = time.perf_counter() - t0
    out["dataset_particle_steps"] = float(n_train) * wl.n_obs * train_particles * wl.n_steps
    if dump:
        np.savez(dump, U=U, G=G, y=y, g_star=g_star, u_star=setup["u_star"], prior_std=prior_std, beta=beta,
                 pilot=np.array(pc.samples))
    if dataset_only:
        prob.close()
        ctx.close()
        return out
    sur = Surrogate(ctx, prior_std, wl.n_obs, seed=seed)
    hist = sur.fit(U, G, epochs=epochs, batch=1024, lr=1e-3)
    out["train_s"] = hist["seconds"]
    out["train_steps"] = hist["steps"]
    out["val_rmse_standardised"] = hist["val_rmse"][-1]
    out["val_rmse_G"] = float(np.sqrt(np.mean((sur.predict(U[hist["val_idx"]]) - G[hist["val_idx"]]) ** 2)))
    out["surrogate_err_at_ustar"] = float(np.sqrt(np.mean((sur(setup["u_star"]) - g_star) ** 2)))
    if verbose:
        print(f"[da] beta {beta}, dataset {out['dataset_s']:.1f} s, training {out['train_s']:.1f} s, "
              f"val rmse {out['val_rmse_G']:.4f} (std units {out['val_rmse_standardised']:.3f})", flush=True)

    coords = list(range(8))
    res = {}
    for kind in ("plain", "da", "da_aem"):
        fwd.calls, fwd.seconds = 0, 0.0
        sur_calls = [0]

        def surf(u):
            sur_calls[0] += 1
            return sur(u)

        gamma_s = np.sqrt(gamma ** 2 + sur.err_std ** 2) if kind == "da_aem" else None
        c = mcmc.start_chain(setup["u_star"], fwd, y, gamma, seed=seed + 2,
                             surrogate=surf if kind != "plain" else None, gamma_s=gamma_s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < iters:  # blocks of 500 iterations with a progress line
            nb = min(500, iters - done)
            if kind == "plain":
                mcmc.pcn_steps(c, nb, fwd, prior_std, y, gamma, beta)
            else:
                mcmc.da_pcn_steps(c, nb, fwd, surf, prior_std, y, gamma, beta, gamma_s=gamma_s)
            done += nb
            if verbose:
                print(f"[da] {kind}: {done}/{iters} iterations, {time.perf_counter() - t0:.1f} s", flush=True)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        S = np.array(c.samples)
        e = mcmc.ess_min(S, coords)
        e_phi = mcmc.ess(np.array(c.phis))
        res[kind] = {"seconds": sec, "samples_per_s": iters / sec, "particle_map_calls": c.n_forward,
                     "accept_rate": c.n_accept / iters, "stage1_pass_rate": c.n_stage1 / iters,
                     "ess_min_first8": e, "ess_phi": e_phi, "ess_per_s": e / sec, "ess_phi_per_s": e_phi / sec,
                     "surrogate_calls": sur_calls[0]}
        if verbose:
            print(f"[da] {kind}: {res[kind]}", flush=True)
    out.update(res)
    for kind in ("da", "da_aem"):
        out[f"{kind}_speedup_samples_per_s"] = res[kind]["samples_per_s"] / res["plain"]["samples_per_s"]
        out[f"{kind}_speedup_ess_per_s"] = (res[kind]["ess_per_s"] / res["plain"]["ess_per_s"]
                                            if res["plain"]["ess_per_s"] > 0 else None)
        out[f"{kind}_speedup_ess_phi_per_s"] = (res[kind]["ess_phi_per_s"] / res["plain"]["ess_phi_per_s"]
                                                if res["plain"]["ess_phi_per_s"] > 0 else None)
    prob.close()
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=8192)
    ap.add_argument("--train-particles", type=int, default=10_000)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--dump", default=None, help="save the training set (npz) here")
    ap.add_argument("--dataset-only", action="store_true", help="stop after the training set")
    ap.add_argument("--horizon", type=float, default=None, help="observation time T (default: the workload's)")
    ap.add_argument("--engine", default="auto", choices=["auto", "valu", "mfma"])
    a = ap.parse_args()
    print(json.dumps(run(a.n_train, a.train_particles, a.iters, epochs=a.epochs, dump=a.dump,
                         dataset_only=a.dataset_only, horizon=a.horizon, engine=a.engine)))


if __name__ == "__main__":
    main()
