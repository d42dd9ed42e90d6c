"""Seeded synthetic inputs for the particle forward map.

This module only draws and lays out inputs (wavevector tables, prior draws of
the unknown u, observation points, initial/boundary/source field descriptors,
particle counts and seeds). It holds none of the method's arithmetic, so both
the CPU oracle and the HIP library may consume what it produces.

Problem data follow the paper's constant-diffusion advection-diffusion example
(Section 4.1, eq. adr, with sigma = sqrt(2 kappa) I) and the Dirichlet problem
(Problem 2.2).  The unknown u is the stream function
    psi(x) = sum_{k in H} a_k cos(2 pi k.x) + b_k sin(2 pi k.x)
stored as u = [a_0 .. a_{M-1}, b_0 .. b_{M-1}] in wavevector-table order; the
velocity is v = (d psi/dy, -d psi/dx), which is the paper's divergence-free
Fourier expansion (eq. v_expand) written over a half-plane of wavevectors.

Field descriptors are dicts {"kind": name, "params": [floats]}; the kinds and
their formulas are listed in FIELD_KINDS.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

WORKLOAD_SEED = 1808

# name -> (number of params per term, description); "n" terms allowed when >0
FIELD_KINDS = {
    "zero": "f(x) = 0",
    "const": "f(x) = c                                  params [c]",
    "sinsin": "f(x) = A sin(2 pi x) sin(2 pi y)          params [A]",
    "fourier": "f(x) = sum_m c_m cos(2pi(p_m x + q_m y)) + d_m sin(2pi(p_m x + q_m y))   params [p,q,c,d]*n",
    "gauss_periodic": "f(x) = sum_m A_m sum_{n in {-1,0,1}^2} exp(-|x - c_m - n|^2 / (2 s_m^2))   params [cx,cy,s,A]*n",
    "cos_m_theta": "f(x) = cos(m * atan2(y, x))                params [m]",
    "exp_linear": "f(x) = exp(c0 x + c1 y)                    params [c0,c1]",
    "linear": "f(x) = c0 x + c1 y + c2                    params [c0,c1,c2]",
    "gauss": "f(x) = sum_m A_m exp(-w_m |x - c_m|^2)      params [cx,cy,w,A]*n",
    "cos_axes": "f(x) = A (cos(w x) + cos(w y))             params [A, w]",
}


def fld(kind: str, params=()) -> dict:
    if kind not in FIELD_KINDS:
        raise ValueError(f"unknown field kind {kind!r}")
    return {"kind": kind, "params": [float(p) for p in params]}


# ----------------------------------------------------------------------------
# Wavevector tables
# ----------------------------------------------------------------------------

def torus_modes(K: int) -> np.ndarray:
    """Half-plane set H_K = {k : 0<=kx<=K, -K<=ky<=K, kx>0 or ky>0} (|k|_inf <= K).

    One representative of each +-k pair, since cos/sin of 2 pi (-k).x carry no
    new functions. |H_2| = 12 (24 coefficients), |H_6| = 84 (168 coefficients).
    """
    out = []
    for kx in range(0, K + 1):
        for ky in range(-K, K + 1):
            if kx == 0 and ky <= 0:
                continue
            out.append((kx, ky))
    return np.asarray(out, dtype=np.int32).reshape(-1, 2)


def disk_modes() -> np.ndarray:
    """32 wavevectors {1<=kx<=4, 1<=|ky|<=4}: a 64-coefficient series for the disk workload."""
    out = [(kx, ky) for kx in range(1, 5) for ky in list(range(-4, 0)) + list(range(1, 5))]
    return np.asarray(out, dtype=np.int32)


def l2_ball_modes(R: float) -> np.ndarray:
    """All k in Z^2 with |k|_2 <= R, including k = 0 (the paper's N_u counting)."""
    r = int(math.floor(R))
    out = [(kx, ky) for kx in range(-r, r + 1) for ky in range(-r, r + 1)
           if kx * kx + ky * ky <= R * R]
    return np.asarray(out, dtype=np.int32)


def prior_std(modes: np.ndarray) -> np.ndarray:
    """Prior standard deviation |k|_2^-2 per mode (variance |k|_2^-4)."""
    k2 = (modes.astype(np.float64) ** 2).sum(axis=1)
    if np.any(k2 == 0):
        raise ValueError("the prior is undefined for k = 0")
    return 1.0 / k2


def draw_prior(modes: np.ndarray, rng: np.random.Generator, n: Optional[int] = None) -> np.ndarray:
    """u = [a, b] with a_k, b_k ~ N(0, |k|^-4) independently."""
    s = prior_std(modes)
    shape = (2 * len(modes),) if n is None else (n, 2 * len(modes))
    z = rng.standard_normal(shape)
    return z * np.concatenate([s, s])


def pcn_proposals(u0: np.ndarray, modes: np.ndarray, beta: float, n: int,
                  rng: np.random.Generator) -> np.ndarray:
    """n proposals sqrt(1-beta^2) u0 + beta xi with xi drawn from the prior."""
    xi = draw_prior(modes, rng, n)
    return math.sqrt(1.0 - beta * beta) * u0[None, :] + beta * xi


# ----------------------------------------------------------------------------
# Observation points
# ----------------------------------------------------------------------------

def grid_points(n: int) -> np.ndarray:
    """Cell centres ((a+1/2)/n, (b+1/2)/n), a,b = 0..n-1, row-major in (a, b)."""
    c = (np.arange(n) + 0.5) / n
    return np.asarray([(x, y) for x in c for y in c], dtype=np.float64)


def uniform_torus_points(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.random((n, 2))


def uniform_disk_points(n: int, r_max: float, rng: np.random.Generator) -> np.ndarray:
    """Uniform in the disk of radius r_max: r = r_max sqrt(U1), phi = 2 pi U2."""
    u = rng.random((n, 2))
    r = r_max * np.sqrt(u[:, 0])
    ph = 2.0 * np.pi * u[:, 1]
    return np.stack([r * np.cos(ph), r * np.sin(ph)], axis=1)


def log_uniform_counts(n: int, lo: float, hi: float, rng: np.random.Generator) -> np.ndarray:
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n))).astype(np.int64)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    domain: str                      # "torus" | "disk"
    modes: np.ndarray                # [M,2] int32
    u: np.ndarray                    # [2M] or [n_u, 2M] float64
    obs: np.ndarray                  # [n_obs,2] float64
    kappa: float
    dt: float
    n_particles: object              # int, or [n_u] int64 for batches
    seed: object                     # int, or [n_u] uint64 for batches
    prec: str                        # "fp32" | "fp64"
    T: Optional[float] = None        # time problem
    theta0: Optional[dict] = None    # time problem
    f: Optional[dict] = None         # Dirichlet
    g: Optional[dict] = None         # Dirichlet
    max_steps: Optional[int] = None  # Dirichlet
    v0: tuple = (0.0, 0.0)           # constant drift added to the Fourier field
    extra: Dict = field(default_factory=dict)

    @property
    def n_obs(self) -> int:
        return int(self.obs.shape[0])

    @property
    def n_steps(self) -> int:
        assert self.T is not None
        return int(math.ceil(self.T / self.dt - 1e-9))


def _gauss_bumps(n: int, sigma: float, rng) -> dict:
    c = rng.random((n, 2))
    params = []
    for m in range(n):
        params += [c[m, 0], c[m, 1], sigma, 1.0]
    return fld("gauss_periodic", params)


def time_small(seed: int = WORKLOAD_SEED) -> Workload:
    """Torus, |k|_inf<=2 (24 coefficients), kappa 0.05, theta0 = sin sin, 4 uniform
    points x 1000 particles, T = 0.1, dt = 1e-3, FP64."""
    rng = np.random.default_rng([seed, 1])
    modes = torus_modes(2)
    u = draw_prior(modes, rng)
    obs = uniform_torus_points(4, rng)
    return Workload("torus-k2-fp64", "torus", modes, u, obs, kappa=0.05, dt=1e-3,
                    n_particles=1000, seed=1, prec="fp64", T=0.1, theta0=fld("sinsin", [1.0]))


def time_main(seed: int = WORKLOAD_SEED, n_particles: int = 100_000) -> Workload:
    """Torus, |k|_inf<=6 (168 coefficients), kappa 0.01, theta0 = 3 periodised
    Gaussian bumps (sigma 0.1), 7x7 grid x 1e5 particles, T = 1, dt = 1e-3, FP32."""
    rng = np.random.default_rng([seed, 2])
    modes = torus_modes(6)
    u = draw_prior(modes, rng)
    theta0 = _gauss_bumps(3, 0.1, rng)
    obs = grid_points(7)
    return Workload("torus-k6-fp32", "torus", modes, u, obs, kappa=0.01, dt=1e-3,
                    n_particles=n_particles, seed=2, prec="fp32", T=1.0, theta0=theta0)


def dirichlet_main(seed: int = WORKLOAD_SEED, n_particles: int = 50_000,
                   prec: str = "fp32") -> Workload:
    """Unit disk, psi = (1-|x|^2)^2 * (64-coefficient Fourier series), kappa 0.02,
    g = cos 3 theta, 25 uniform points in r<=0.8 x 5e4 particles, dt = 1e-4.

    The workload reads g(X_tau) + int_0^tau 1 ds.  Theorem 3.2's payoff is
    g(X_tau) - int f, so that output is the paper's theta with source f = -1."""
    rng = np.random.default_rng([seed, 3])
    modes = disk_modes()
    u = draw_prior(modes, rng)
    obs = uniform_disk_points(25, 0.8, rng)
    return Workload("disk-dirichlet", "disk", modes, u, obs, kappa=0.02, dt=1e-4,
                    n_particles=n_particles, seed=3, prec=prec, f=fld("const", [-1.0]),
                    g=fld("cos_m_theta", [3.0]), max_steps=20_000_000)


def batch_main(seed: int = WORKLOAD_SEED, n_u: int = 512, lo: float = 1e3,
               hi: float = 1e5) -> Workload:
    """512 pCN proposals (beta = 0.2) around a prior draw of the |k|_inf<=6 torus
    problem, per-u particle counts log-uniform in [1e3, 1e5], FP32."""
    base = time_main(seed)
    rng = np.random.default_rng([seed, 4])
    u0 = draw_prior(base.modes, rng)
    U = pcn_proposals(u0, base.modes, 0.2, n_u, rng)
    counts = log_uniform_counts(n_u, lo, hi, rng)
    seeds = (1000 + np.arange(n_u)).astype(np.uint64)
    return Workload("torus-k6-batch", "torus", base.modes, U, base.obs, kappa=base.kappa,
                    dt=base.dt, n_particles=counts, seed=seeds, prec="fp32", T=base.T,
                    theta0=base.theta0, extra={"u0": u0, "beta": 0.2})


def half_plane(modes: np.ndarray) -> np.ndarray:
    """One representative of each +-k pair (k_x > 0, or k_x = 0 and k_y > 0); k = 0 dropped."""
    keep = [(kx, ky) for kx, ky in modes if kx > 0 or (kx == 0 and ky > 0)]
    return np.asarray(keep, dtype=np.int32).reshape(-1, 2)


def turbulent_k80(seed: int = WORKLOAD_SEED, n_particles: int = 100_000) -> Workload:
    """The regime of the paper's turbulent example: |k|_2 <= 80 (20,081 modes
    counting k = 0 and both signs; 10,040 half-plane modes, 20,080
    coefficients), kappa 3e-5, observed at 13 evenly spaced times in [0, 0.5]
    at (0, 0) and (1/2, 1/2).  The paper does not give theta0 or the prior for
    it: theta0 is 3 periodised Gaussian bumps (sigma 0.1) and the prior is the
    |k|^-4 variance of the other workloads.  dt = 1/9600 puts every observation
    time on the step grid (t_k = 400 k dt, 4,800 steps to T = 0.5).  FP32."""
    rng = np.random.default_rng([seed, 7])
    modes = half_plane(l2_ball_modes(80.0))
    u = draw_prior(modes, rng)
    theta0 = _gauss_bumps(3, 0.1, rng)
    obs = np.array([[0.0, 0.0], [0.5, 0.5]])
    dt = 1.0 / 9600.0
    reads = (400 * np.arange(13)).astype(np.int64)
    return Workload("torus-k80-turbulent", "torus", modes, u, obs, kappa=3e-5, dt=dt,
                    n_particles=n_particles, seed=7, prec="fp32", T=0.5, theta0=theta0,
                    extra={"read_steps": reads})


def bvp_square(seed: int = WORKLOAD_SEED, n_particles: int = 100_000) -> Workload:
    """The paper's optimal-forcing example (Problem 2.2 on the unit square):
    -(1,1).grad theta + kappa Lap theta = sum_j f_j exp(-4 |x - x_f^(j)|^2),
    theta = (cos(pi x / 2) + cos(pi y / 2)) / 2 on the boundary, kappa = 0.282,
    three observation points, data y = [0, 0, 0].  The forcing and observation
    locations appear only in a figure of the paper: here they are seeded
    uniform draws in [0.15, 0.85]^2.  dt = 1e-4, 1e5 particles per point."""
    rng = np.random.default_rng([seed, 8])
    sources = [(float(cx), float(cy), 4.0) for cx, cy in 0.15 + 0.7 * rng.random((3, 2))]
    obs = 0.15 + 0.7 * rng.random((3, 2))
    return Workload("square-bvp", "square", np.zeros((0, 2), dtype=np.int32), np.zeros(0), obs, kappa=0.282,
                    dt=1e-4, n_particles=n_particles, seed=8, prec="fp64", v0=(1.0, 1.0),
                    g=fld("cos_axes", [0.5, math.pi / 2]), max_steps=10_000_000,
                    extra={"sources": sources, "data": np.zeros(3)})


def surrogate_setup(seed: int = WORKLOAD_SEED) -> dict:
    """Inputs of the delayed-acceptance study: the true parameter u*, the noise level
    and the standard-normal draws that make the synthetic data y = G(u*) + gamma*eta."""
    base = time_main(seed)
    rng = np.random.default_rng([seed, 5])
    u_star = draw_prior(base.modes, rng)
    eta = rng.standard_normal(base.n_obs)
    return {"base": base, "u_star": u_star, "gamma": 0.01, "eta": eta}


WORKLOADS = {
    "torus-k2-fp64": time_small,
    "torus-k6-fp32": time_main,
    "disk-dirichlet": dirichlet_main,
    "torus-k6-batch": batch_main,
    "torus-k80-turbulent": turbulent_k80,
    "square-bvp": bvp_square,
}
