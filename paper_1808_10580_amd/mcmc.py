"""pCN and delayed-acceptance pCN over the particle forward map.

The paper samples its Bayesian posteriors with preconditioned Crank-Nicolson
MCMC (Section 4.1; Cotter, Roberts, Stuart and White, 2013), one forward map
G(u) per proposal.  For a Gaussian prior N(0, C) the pCN proposal

    v = sqrt(1 - beta^2) u + beta xi,   xi ~ N(0, C),

is prior-reversible, so the Metropolis-Hastings ratio only involves the data
misfit Phi(u) = |y - G(u)|^2 / (2 gamma^2):  accept with probability
min(1, exp(Phi(u) - Phi(v))).

Delayed acceptance (Christen and Fox, 2005) screens each proposal with a cheap
approximation Phi~ (here: a learned surrogate of G) first,

    stage 1: accept with min(1, exp(Phi~(u) - Phi~(v)))
    stage 2: accept with min(1, exp([Phi(u) - Phi(v)] - [Phi~(u) - Phi~(v)])),

running the particle map only for proposals that pass stage 1.  The chain
still targets the exact posterior of the particle map.

Random streams: proposals, stage-1 and stage-2 uniforms come from three
independent generators, so delayed acceptance with Phi~ = 0 reproduces plain
pCN bit for bit.  The forward map uses common random numbers (one Philox seed
for every evaluation), which makes G deterministic in u.

Chains checkpoint to a plain dict (state, generator states, counters) and
resume bit for bit.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np


def misfit(G: np.ndarray, y: np.ndarray, gamma) -> float:
    """Phi = |y - G|^2 / (2 gamma^2) in FP64; gamma may be one value or one
    per observation."""
    r = np.asarray(y, dtype=np.float64) - np.asarray(G, dtype=np.float64)
    if np.ndim(gamma) == 0:
        return float(r @ r) / (2.0 * gamma * gamma)
    g = np.asarray(gamma, dtype=np.float64)
    return float(np.sum(r * r / (2.0 * g * g)))


def _gen(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


@dataclass
class Chain:
    """State of a (delayed-acceptance) pCN chain; ``checkpoint()`` / ``resume()``."""
    u: np.ndarray
    phi: float
    phi_s: float = 0.0
    it: int = 0
    n_stage1: int = 0      # proposals that passed stage 1 (DA) / were evaluated (plain)
    n_accept: int = 0
    n_forward: int = 0     # particle-map evaluations after the initial one
    rng_prop: np.random.Generator = None
    rng_s1: np.random.Generator = None
    rng_s2: np.random.Generator = None
    samples: List[np.ndarray] = field(default_factory=list)
    phis: List[float] = field(default_factory=list)

    def checkpoint(self) -> Dict:
        return {"u": self.u.copy(), "phi": self.phi, "phi_s": self.phi_s, "it": self.it,
                "n_stage1": self.n_stage1, "n_accept": self.n_accept, "n_forward": self.n_forward,
                "rng_prop": self.rng_prop.bit_generator.state, "rng_s1": self.rng_s1.bit_generator.state,
                "rng_s2": self.rng_s2.bit_generator.state}

    @staticmethod
    def resume(ck: Dict) -> "Chain":
        c = Chain(u=np.array(ck["u"], dtype=np.float64), phi=float(ck["phi"]), phi_s=float(ck["phi_s"]),
                  it=int(ck["it"]), n_stage1=int(ck["n_stage1"]), n_accept=int(ck["n_accept"]),
                  n_forward=int(ck["n_forward"]))
        for name in ("rng_prop", "rng_s1", "rng_s2"):
            g = np.random.Generator(np.random.PCG64())
            g.bit_generator.state = ck[name]
            setattr(c, name, g)
        return c


def start_chain(u0, forward: Callable, y, gamma: float, seed: int,
                surrogate: Optional[Callable] = None, gamma_s=None) -> Chain:
    """gamma_s: noise level of the stage-1 (surrogate) misfit, default gamma."""
    u0 = np.array(u0, dtype=np.float64)
    c = Chain(u=u0, phi=misfit(forward(u0), y, gamma))
    if surrogate is not None:
        c.phi_s = misfit(surrogate(u0), y, gamma if gamma_s is None else gamma_s)
    c.rng_prop, c.rng_s1, c.rng_s2 = _gen(seed, 0), _gen(seed, 1), _gen(seed, 2)
    return c


def _propose(c: Chain, prior_std: np.ndarray, beta: float) -> np.ndarray:
    xi = c.rng_prop.standard_normal(c.u.shape[0]) * prior_std
    return math.sqrt(1.0 - beta * beta) * c.u + beta * xi


def pcn_steps(c: Chain, n: int, forward: Callable, prior_std, y, gamma: float, beta: float,
              keep_every: int = 1) -> Chain:
    """n plain pCN iterations (one forward map each)."""
    prior_std = np.asarray(prior_std, dtype=np.float64)
    for _ in range(n):
        v = _propose(c, prior_std, beta)
        phi_v = misfit(forward(v), y, gamma)
        c.n_forward += 1
        c.n_stage1 += 1
        log_a = c.phi - phi_v
        if math.log(c.rng_s2.random()) < log_a:
            c.u, c.phi = v, phi_v
            c.n_accept += 1
        c.it += 1
        if keep_every and c.it % keep_every == 0:
            c.samples.append(c.u.copy())
            c.phis.append(c.phi)
    return c


def da_pcn_steps(c: Chain, n: int, forward: Callable, surrogate: Callable, prior_std, y,
                 gamma: float, beta: float, keep_every: int = 1, gamma_s=None) -> Chain:
    """n delayed-acceptance pCN iterations: the surrogate screens, the particle
    map decides.  gamma_s (scalar or per observation; default gamma) is the
    noise level of the stage-1 misfit: widening it by the surrogate's own
    error, gamma_s^2 = gamma^2 + sigma_j^2 (an approximation-error model),
    makes stage 1 reject fewer proposals the particle map would accept.  Any
    gamma_s leaves the chain exact: stage 2 divides the stage-1 ratio out."""
    prior_std = np.asarray(prior_std, dtype=np.float64)
    gs = gamma if gamma_s is None else gamma_s
    for _ in range(n):
        v = _propose(c, prior_std, beta)
        phis_v = misfit(surrogate(v), y, gs)
        log_a1 = c.phi_s - phis_v
        passed = log_a1 >= 0.0 or math.log(c.rng_s1.random()) < log_a1
        if passed:
            c.n_stage1 += 1
            phi_v = misfit(forward(v), y, gamma)
            c.n_forward += 1
            log_a2 = (c.phi - phi_v) - (c.phi_s - phis_v)
            if math.log(c.rng_s2.random()) < log_a2:
                c.u, c.phi, c.phi_s = v, phi_v, phis_v
                c.n_accept += 1
        c.it += 1
        if keep_every and c.it % keep_every == 0:
            c.samples.append(c.u.copy())
            c.phis.append(c.phi)
    return c


def ess(x: np.ndarray) -> float:
    """Effective sample size of a scalar chain by Geyer's initial monotone
    sequence estimator (Geyer, 1992): sum autocorrelations in adjacent pairs
    while the pair sums stay positive and non-increasing."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 4:
        return float(n)
    x = x - x.mean()
    f = np.fft.rfft(x, 2 * n)
    acov = np.fft.irfft(f * np.conj(f))[:n] / n
    if acov[0] <= 0:
        return float(n)
    rho = acov / acov[0]
    s = 0.0
    prev = np.inf
    for k in range(0, n - 1, 2):
        g = rho[k] + rho[k + 1]
        if g <= 0:
            break
        g = min(g, prev)
        s += g
        prev = g
    tau = -1.0 + 2.0 * s
    return float(n / max(tau, 1e-12))


def ess_min(samples: np.ndarray, coords) -> float:
    samples = np.asarray(samples)
    return min(ess(samples[:, c]) for c in coords)


class ParticleForward:
    """G(u) by the particle map: a captured graph replay (u rewritten in place)
    with common random numbers; returns the 49 means on the host."""

    def __init__(self, problem, wl, n_particles: int, seed: int, use_graph: bool = True):
        import torch
        self.problem = problem
        self.u_dev = torch.tensor(np.zeros(2 * len(wl.modes)), dtype=torch.float64, device="cuda")
        self.obs = torch.tensor(wl.obs, dtype=torch.float64, device="cuda")
        self.wl = wl
        self.n_particles = int(n_particles)
        self.seed = int(seed)
        self.graph = (problem.graph_time(self.u_dev, self.obs, wl.kappa, wl.T, wl.dt, n_particles, seed)
                      if use_graph else None)
        self.calls = 0
        self.seconds = 0.0

    def __call__(self, u) -> np.ndarray:
        import torch
        t0 = time.perf_counter()
        self.u_dev.copy_(torch.as_tensor(np.asarray(u, dtype=np.float64)))
        if self.graph is not None:
            m, _ = self.graph.replay()
        else:
            m, _ = self.problem.observe_time(self.u_dev, self.obs, self.wl.kappa, self.wl.T, self.wl.dt,
                                             self.n_particles, self.seed)
        out = m.cpu().numpy()
        self.calls += 1
        self.seconds += time.perf_counter() - t0
        return out
