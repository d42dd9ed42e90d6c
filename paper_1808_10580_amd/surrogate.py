"""Learned surrogate of the forward map G(u) (first stage of delayed-acceptance pCN).

Training pairs (u, G(u)) come from the particle map itself: u drawn from the
prior, G evaluated with the batched persistent kernel (pm_observe_time_batch)
at a reduced particle count.  The network (include/pm_mlp.h) sees whitened
inputs u / prior_std and standardised outputs; its training and inference run
on the GPU through libpm's BF16 MFMA kernels.
"""
from __future__ import annotations

import math
import time
from typing import Dict, Optional

import numpy as np

import paper_1808_10580_amd as pm


def particle_dataset(problem, wl, U: np.ndarray, n_particles: int, seed: int, chunk: int = 512,
                     progress=None) -> np.ndarray:
    """G(u) for every row of U with the batched particle map (common random
    numbers: one Philox seed for every evaluation).  progress(done, total) is
    called after each launch when given."""
    out = []
    for s in range(0, U.shape[0], chunk):
        Ub = U[s:s + chunk]
        nb = Ub.shape[0]
        m, _ = problem.observe_time_batch(Ub, [n_particles] * nb, [seed] * nb, wl.obs, wl.kappa, wl.T, wl.dt)
        out.append(m.cpu().numpy())
        if progress is not None:
            progress(s + nb, U.shape[0])
    problem.ctx.sync(raise_on_flags=True)
    return np.concatenate(out, axis=0)


class Surrogate:
    def __init__(self, ctx: pm.Context, prior_std: np.ndarray, d_out: int, d_hidden: int = 512,
                 n_hidden: int = 3, max_batch: int = 1024, seed: int = 0):
        self.d_in = int(prior_std.size)
        self.d_out = d_out
        self.net = pm.MLP(ctx, self.d_in, d_hidden, n_hidden, d_out, max_batch, seed)
        self.net.set_io(in_scale=1.0 / np.asarray(prior_std, dtype=np.float64))
        self.max_batch = max_batch

    def fit(self, U: np.ndarray, G: np.ndarray, epochs: int = 20, batch: int = 1024, lr: float = 1e-3,
            holdout: float = 0.1, seed: int = 0, lr_final: Optional[float] = None, progress=None,
            early_stop: bool = False) -> Dict:
        """Adam on the standardised MSE; the learning rate decays geometrically
        from lr to lr_final over the epochs when lr_final is given.
        progress(epoch, val_rmse) is called after each epoch when given.
        early_stop: keep the parameters of the epoch with the lowest held-out
        error (the held-out rows are then also the selection set)."""
        import torch
        rng = np.random.default_rng(seed)
        n = U.shape[0]
        idx = rng.permutation(n)
        n_val = max(1, int(round(holdout * n)))
        val, tr = idx[:n_val], idx[n_val:]
        mu = G[tr].mean(axis=0)
        sd = G[tr].std(axis=0) + 1e-12
        self.net.set_io(out_mean=mu, out_std=sd)
        self.out_mean, self.out_std = mu, sd
        dev = self.net.ctx.device
        Ut = torch.tensor(U[tr], dtype=torch.float32, device=dev)
        Gt = torch.tensor(G[tr], dtype=torch.float32, device=dev)
        hist = {"train": [], "val_rmse": [], "seconds": 0.0, "steps": 0}
        t0 = time.perf_counter()
        b = min(batch, self.max_batch)
        for ep in range(epochs):
            lr_ep = lr if lr_final is None or epochs < 2 else lr * (lr_final / lr) ** (ep / (epochs - 1))
            perm = torch.randperm(Ut.shape[0], device=dev)
            losses = []
            for s in range(0, Ut.shape[0] - b + 1, b):
                sel = perm[s:s + b]
                loss = self.net.train_step(Ut[sel], Gt[sel], lr_ep)
                losses.append(loss.clone())
                hist["steps"] += 1
            hist["train"].append(float(torch.stack(losses).mean().item()) if losses else float("nan"))
            pv = self.predict(U[val])
            hist["val_rmse"].append(float(np.sqrt(np.mean(((pv - G[val]) / sd) ** 2))))
            if early_stop and hist["val_rmse"][-1] <= min(hist["val_rmse"]):
                best = (ep, self.net.get_params())
            if progress is not None:
                progress(ep, hist["val_rmse"][-1])
        if early_stop and epochs > 0:
            hist["best_epoch"] = best[0]
            self.net.set_params(best[1])  # also resets the Adam moments
        torch.cuda.synchronize()
        hist["seconds"] = time.perf_counter() - t0
        hist["val_idx"] = val
        # held-out error per observation (physical units): the approximation
        # error a delayed-acceptance stage 1 can add to the data noise
        pv = self.predict(U[val])
        self.err_std = np.sqrt(np.mean((pv - G[val]) ** 2, axis=0))
        hist["err_std"] = self.err_std
        return hist

    def state(self) -> Dict:
        """Everything needed to rebuild the fitted network (host arrays)."""
        return {"params": self.net.get_params(), "out_mean": self.out_mean, "out_std": self.out_std,
                "err_std": self.err_std}

    def load(self, st: Dict) -> "Surrogate":
        self.net.set_params(np.asarray(st["params"], dtype=np.float32))
        self.out_mean = np.asarray(st["out_mean"], dtype=np.float64)
        self.out_std = np.asarray(st["out_std"], dtype=np.float64)
        self.err_std = np.asarray(st["err_std"], dtype=np.float64)
        self.net.set_io(out_mean=self.out_mean, out_std=self.out_std)
        return self

    def predict(self, U: np.ndarray) -> np.ndarray:
        U = np.atleast_2d(np.asarray(U, dtype=np.float64))
        out = []
        for s in range(0, U.shape[0], self.max_batch):
            out.append(self.net.forward(U[s:s + self.max_batch]).cpu().numpy().astype(np.float64))
        return np.concatenate(out, axis=0)

    def __call__(self, u) -> np.ndarray:
        return self.predict(np.asarray(u)[None, :])[0]
