"""Optimal forcing for the Dirichlet problem on the unit square (the paper's
boundary-value example, Section 4).

    python -m paper_1808_10580_amd.forcing [--particles 100000]

The paper minimises |y - G(F)| over the weights F of three Gaussian sources
with Nelder-Mead, running the particle method for every evaluation of G
(thousands of them).  By Theorem 3.2 the solution at an observation point is
E[theta_dD(X_tau)] - sum_q f_q E[int phi_q(X_t) dt], so on common random
numbers G(F) = a - B^T F is affine in F: one particle run that records one
integral per source along each path (pm_observe_dirichlet_sources) gives G
for every F.  The optimiser then runs on that affine map (Nelder-Mead as in
the paper, and the exact least-squares solution for comparison), and a final
particle run with the optimal source checks the result.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def affine_map(prob, wl, n_particles=None, seed=None):
    """(a, B) with G(F) = a - B^T F, B [n_src, n_obs], from one GPU run."""
    out = prob.observe_dirichlet_sources(wl.u, wl.g, wl.obs, wl.kappa, wl.dt, n_particles or wl.n_particles,
                                         seed if seed is not None else wl.seed, wl.max_steps, wl.extra["sources"])
    return out["bnd_mean"].cpu().numpy(), out["B"].cpu().numpy(), out


def optimal_forcing(a, B, y, x0=None):
    """Nelder-Mead on |y - (a - B^T F)| (the paper's optimiser on the affine map)
    and the least-squares solution; returns both and the evaluation count."""
    from scipy.optimize import minimize

    def cost(F):
        return float(np.linalg.norm(y - (a - B.T @ F)))
    x0 = np.zeros(B.shape[0]) if x0 is None else x0
    res = minimize(cost, x0, method="Nelder-Mead", options={"xatol": 1e-10, "fatol": 1e-12, "maxiter": 20000,
                                                            "maxfev": 40000})
    F_ls, *_ = np.linalg.lstsq(-B.T, y - a, rcond=None)
    return {"F_nm": res.x, "cost_nm": res.fun, "evals_nm": int(res.nfev), "F_ls": F_ls, "cost_ls": cost(F_ls)}


def run(n_particles=100_000, verbose=True):
    import torch

    import paper_1808_10580_amd as pm
    import workloads as W

    wl = W.bvp_square(n_particles=n_particles)
    y = wl.extra["data"]
    ctx = pm.Context(0)
    prob = pm.Problem(ctx, "square", wl.modes, v0=wl.v0, prec=wl.prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, B, raw = affine_map(prob, wl)
    ctx.sync(raise_on_flags=True)
    t_map = time.perf_counter() - t0
    steps = float(raw["tau_mean"].cpu().numpy().sum() / wl.dt * wl.n_particles)
    opt = optimal_forcing(a, B, y)
    # check: a direct particle run with the optimal source, same seed
    F = opt["F_nm"]
    f = {"kind": "gauss", "params": [v for (cx, cy, w), fq in zip(wl.extra["sources"], F) for v in (cx, cy, w, fq)]}
    chk = prob.observe_dirichlet(wl.u, f, wl.g, wl.obs, wl.kappa, wl.dt, wl.n_particles, wl.seed, wl.max_steps)
    G_chk = chk["mean"].cpu().numpy()
    out = {"n_particles": n_particles, "affine_map_s": t_map, "particle_steps": steps,
           "a": a.tolist(), "B": B.tolist(), "F_nelder_mead": F.tolist(), "nm_evaluations": opt["evals_nm"],
           "cost_nm": opt["cost_nm"], "F_least_squares": opt["F_ls"].tolist(), "cost_ls": opt["cost_ls"],
           "G_check": G_chk.tolist(), "G_affine": (a - B.T @ F).tolist(),
           "check_se": np.sqrt(chk["var"].cpu().numpy() / wl.n_particles).tolist()}
    if verbose:
        print(f"[forcing] affine map {t_map:.3f} s ({steps:.3g} particle-steps); Nelder-Mead "
              f"{opt['evals_nm']} evaluations on it, F = {np.round(F, 4)}, |y - G| = {opt['cost_nm']:.2e}",
              flush=True)
    prob.close()
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--particles", type=int, default=100_000)
    a = ap.parse_args()
    print(json.dumps(run(a.particles)))


if __name__ == "__main__":
    main()
