"""FP64 CPU oracle of the particle forward map (ctypes front end of pm_oracle.c).

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The HIP library and
its Python binding never import it, and it imports nothing from them.

Every function states the passage of the paper it follows; the arithmetic
lives in pm_oracle.c (paths, velocity, fields, Philox/Box-Muller) and, for the
per-observation statistics, in ``mean_var`` below (the plain definitions of the
sample mean and the unbiased sample variance).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pm_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

FIELD_CODES = {"zero": 0, "const": 1, "sinsin": 2, "fourier": 3, "gauss_periodic": 4,
               "cos_m_theta": 5, "exp_linear": 6, "linear": 7, "gauss": 8, "cos_axes": 9}
DOMAIN_CODES = {"torus": 0, "disk": 1, "square": 2}


def build(force: bool = True) -> str:
    """Compile pm_oracle.c into oracle/_build/liboracle.so (plain gcc, OpenMP)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_params", C.c_int), ("p", C.POINTER(C.c_double))]


class _Flow(C.Structure):
    _fields_ = [("domain", C.c_int), ("n_modes", C.c_int), ("k", C.POINTER(C.c_int32)),
                ("u", C.POINTER(C.c_double)), ("v0", C.c_double * 2)]


_dp = C.POINTER(C.c_double)
_u64p = C.POINTER(C.c_uint64)
_u32p = C.POINTER(C.c_uint32)
_i64p = C.POINTER(C.c_int64)
_u8p = C.POINTER(C.c_uint8)


def _declare(L):
    L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.orc_normals_many.argtypes = [C.c_uint64, C.c_int64, _u64p, _u32p, _u32p, _dp]
    L.orc_field_many.argtypes = [C.POINTER(_Field), C.c_int64, _dp, _dp]
    L.orc_velocity_many.argtypes = [C.POINTER(_Flow), C.c_int64, _dp, _dp]
    L.orc_psi_many.argtypes = [C.POINTER(_Flow), C.c_int64, _dp, _dp]
    L.orc_step.argtypes = [C.POINTER(_Flow), C.c_double, C.c_double, C.c_uint64, C.c_int64,
                           _dp, _u64p, _u32p, _u32p, _dp]
    L.orc_n_steps.argtypes = [C.c_double, C.c_double]
    L.orc_n_steps.restype = C.c_int64
    L.orc_path.argtypes = [C.POINTER(_Flow), C.c_double, C.c_double, C.c_uint64, C.c_uint32,
                           C.c_uint32, _dp, C.c_int64, _dp]
    L.orc_observe_time.argtypes = [C.POINTER(_Flow), C.POINTER(_Field), _dp, C.c_int, C.c_double,
                                   C.c_double, C.c_double, C.c_int64, C.c_uint64, _dp, _dp]
    L.orc_observe_time_steps.argtypes = [C.POINTER(_Flow), C.POINTER(_Field), _dp, C.c_int,
                                         C.c_double, C.c_double, C.c_int64, C.c_int64, C.c_uint64,
                                         _dp, _dp]
    L.orc_observe_dirichlet.argtypes = [C.POINTER(_Flow), C.POINTER(_Field), C.POINTER(_Field),
                                        _dp, C.c_int, C.c_double, C.c_double, C.c_int64,
                                        C.c_uint64, C.c_int64, _dp, _i64p, _u8p, _dp]
    L.orc_num_threads.restype = C.c_int


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class _Keep:
    """Holds numpy buffers alive for the duration of a call."""

    def __init__(self):
        self.items = []

    def arr(self, x, dtype):
        a = np.ascontiguousarray(x, dtype=dtype)
        self.items.append(a)
        return a


def _field(keep: _Keep, fd: Optional[dict]):
    if fd is None:
        fd = {"kind": "zero", "params": []}
    p = keep.arr(np.asarray(fd.get("params", []), dtype=np.float64).reshape(-1), np.float64)
    if p.size == 0:
        p = keep.arr(np.zeros(1), np.float64)
    f = _Field(FIELD_CODES[fd["kind"]], len(fd.get("params", [])), _ptr(p, C.c_double))
    keep.items.append(f)
    return f


def _flow(keep: _Keep, domain: str, modes, u, v0=(0.0, 0.0)):
    modes = np.asarray(modes, dtype=np.int32).reshape(-1, 2)
    M = modes.shape[0]
    k = keep.arr(modes if M else np.zeros((1, 2), np.int32), np.int32)
    uu = np.asarray(u, dtype=np.float64).reshape(-1)
    if uu.size != 2 * M:
        raise ValueError(f"u has {uu.size} entries, expected {2 * M}")
    ua = keep.arr(uu if M else np.zeros(2), np.float64)
    fl = _Flow(DOMAIN_CODES[domain], M, _ptr(k, C.c_int32), _ptr(ua, C.c_double),
               (C.c_double * 2)(float(v0[0]), float(v0[1])))
    keep.items.append(fl)
    return fl


# ---------------------------------------------------------------------------
# Random numbers
# ---------------------------------------------------------------------------

def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block function (SC'11), one 4-word counter, 2-word key."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def normals(seed: int, n, i, j) -> np.ndarray:
    """Normal pairs xi for steps n of particles (i, j): [count, 2]."""
    n = np.ascontiguousarray(np.atleast_1d(n), dtype=np.uint64)
    i = np.ascontiguousarray(np.broadcast_to(np.asarray(i, dtype=np.uint32), n.shape))
    j = np.ascontiguousarray(np.broadcast_to(np.asarray(j, dtype=np.uint32), n.shape))
    z = np.zeros((n.size, 2))
    lib().orc_normals_many(C.c_uint64(int(seed)), n.size, _ptr(n, C.c_uint64),
                           _ptr(i, C.c_uint32), _ptr(j, C.c_uint32), _ptr(z, C.c_double))
    return z


# ---------------------------------------------------------------------------
# Fields, stream function and velocity (Section 4.1, eq. v_expand)
# ---------------------------------------------------------------------------

def field(fd: dict, X) -> np.ndarray:
    keep = _Keep()
    X = keep.arr(np.asarray(X, dtype=np.float64).reshape(-1, 2), np.float64)
    out = np.zeros(X.shape[0])
    f = _field(keep, fd)
    lib().orc_field_many(C.byref(f), X.shape[0], _ptr(X, C.c_double), _ptr(out, C.c_double))
    return out


def velocity(domain: str, modes, u, X, v0=(0.0, 0.0)) -> np.ndarray:
    keep = _Keep()
    X = keep.arr(np.asarray(X, dtype=np.float64).reshape(-1, 2), np.float64)
    V = np.zeros_like(X)
    fl = _flow(keep, domain, modes, u, v0)
    lib().orc_velocity_many(C.byref(fl), X.shape[0], _ptr(X, C.c_double), _ptr(V, C.c_double))
    return V


def stream(domain: str, modes, u, X) -> np.ndarray:
    keep = _Keep()
    X = keep.arr(np.asarray(X, dtype=np.float64).reshape(-1, 2), np.float64)
    P = np.zeros(X.shape[0])
    fl = _flow(keep, domain, modes, u)
    lib().orc_psi_many(C.byref(fl), X.shape[0], _ptr(X, C.c_double), _ptr(P, C.c_double))
    return P


# ---------------------------------------------------------------------------
# Paths (eq. euler) and the two algorithms
# ---------------------------------------------------------------------------

def n_steps(T: float, dt: float) -> int:
    return int(lib().orc_n_steps(T, dt))


def step(domain, modes, u, kappa, dt, seed, X, n, i, j, v0=(0.0, 0.0)) -> np.ndarray:
    """Teacher-forced EM steps (eq. euler): X[e] -> X_{n[e]+1} of particle (i[e], j[e])."""
    keep = _Keep()
    X = keep.arr(np.asarray(X, dtype=np.float64).reshape(-1, 2), np.float64)
    cnt = X.shape[0]
    n = keep.arr(np.broadcast_to(np.asarray(n, dtype=np.uint64), (cnt,)), np.uint64)
    i = keep.arr(np.broadcast_to(np.asarray(i, dtype=np.uint32), (cnt,)), np.uint32)
    j = keep.arr(np.broadcast_to(np.asarray(j, dtype=np.uint32), (cnt,)), np.uint32)
    Y = np.zeros_like(X)
    fl = _flow(keep, domain, modes, u, v0)
    lib().orc_step(C.byref(fl), kappa, dt, C.c_uint64(int(seed)), cnt, _ptr(X, C.c_double),
                   _ptr(n, C.c_uint64), _ptr(i, C.c_uint32), _ptr(j, C.c_uint32),
                   _ptr(Y, C.c_double))
    return Y


def path(domain, modes, u, kappa, dt_eff, seed, i, j, x0, nsteps, v0=(0.0, 0.0)) -> np.ndarray:
    """Trajectory [nsteps+1, 2] of particle i launched from x0 (observation index j)."""
    keep = _Keep()
    x0 = keep.arr(np.asarray(x0, dtype=np.float64).reshape(2), np.float64)
    out = np.zeros((nsteps + 1, 2))
    fl = _flow(keep, domain, modes, u, v0)
    lib().orc_path(C.byref(fl), kappa, dt_eff, C.c_uint64(int(seed)), int(i), int(j),
                   _ptr(x0, C.c_double), int(nsteps), _ptr(out, C.c_double))
    return out


def observe_time_payoffs(modes, u, theta0, obs, kappa, T, dt, n_particles, seed,
                         v0=(0.0, 0.0), endpoints=False):
    """Algorithm 1: per-particle payoffs theta0(X_T) [n_obs, Np] (and X_T)."""
    keep = _Keep()
    obs = keep.arr(np.asarray(obs, dtype=np.float64).reshape(-1, 2), np.float64)
    n_obs = obs.shape[0]
    pay = np.zeros((n_obs, int(n_particles)))
    ep = np.zeros((n_obs, int(n_particles), 2)) if endpoints else None
    fl = _flow(keep, "torus", modes, u, v0)
    f0 = _field(keep, theta0)
    lib().orc_observe_time(C.byref(fl), C.byref(f0), _ptr(obs, C.c_double), n_obs, kappa, T, dt,
                           int(n_particles), C.c_uint64(int(seed)), _ptr(pay, C.c_double),
                           _ptr(ep, C.c_double) if ep is not None else None)
    return (pay, ep) if endpoints else pay


def observe_time_steps_payoffs(modes, u, theta0, obs, kappa, dt, n_steps_, n_particles, seed,
                               v0=(0.0, 0.0)):
    """Algorithm 1 with n_steps_ Euler-Maruyama steps of size dt: payoffs
    theta0(X_{n dt}) [n_obs, Np] (n_steps_ = 0 reads theta0 at the start)."""
    keep = _Keep()
    obs = keep.arr(np.asarray(obs, dtype=np.float64).reshape(-1, 2), np.float64)
    n_obs = obs.shape[0]
    pay = np.zeros((n_obs, int(n_particles)))
    fl = _flow(keep, "torus", modes, u, v0)
    f0 = _field(keep, theta0)
    lib().orc_observe_time_steps(C.byref(fl), C.byref(f0), _ptr(obs, C.c_double), n_obs, kappa, dt,
                                 int(n_steps_), int(n_particles), C.c_uint64(int(seed)),
                                 _ptr(pay, C.c_double), None)
    return pay


def observe_time_multi(modes, u, theta0, obs, kappa, read_steps, dt, n_particles, seed, v0=(0.0, 0.0)):
    """Observations at several times t_k = read_steps[k] dt: Algorithm 1 run
    once per (t_k, x_j), each with its own ensemble of n_particles paths of
    step dt from the same seed.  Returns (mean, var), each [n_read, n_obs]."""
    ms, vs = [], []
    for n in read_steps:
        m, v = mean_var(observe_time_steps_payoffs(modes, u, theta0, obs, kappa, dt, int(n), n_particles,
                                                   seed, v0))
        ms.append(m)
        vs.append(v)
    return np.array(ms), np.array(vs)


def jacobian_time(modes, u, theta0, obs, kappa, T, dt, n_particles, seed, h, v0=(0.0, 0.0)):
    """Central finite differences of Algorithm 1's G with common random
    numbers (the same seed for every evaluation):
        J[j][k] = (G_j(u + h e_k) - G_j(u - h e_k)) / ((u_k + h) - (u_k - h)).
    Returns J [n_obs, 2M]."""
    u = np.asarray(u, dtype=np.float64)
    n = u.size
    cols = []
    for k in range(n):
        up, um = u.copy(), u.copy()
        up[k] = u[k] + h
        um[k] = u[k] - h
        gp, _ = observe_time(modes, up, theta0, obs, kappa, T, dt, n_particles, seed, v0)
        gm, _ = observe_time(modes, um, theta0, obs, kappa, T, dt, n_particles, seed, v0)
        cols.append((gp - gm) / (up[k] - um[k]))
    return np.stack(cols, axis=1)


def observe_dirichlet_paths(modes, u, f, g, obs, kappa, dt, n_particles, seed, max_steps,
                            v0=(0.0, 0.0), domain="disk"):
    """Algorithm 2 on the unit disk or the unit square: per-particle payoffs,
    exit steps, capped flags and exit points, each [n_obs, Np] (exit points
    [n_obs, Np, 2])."""
    keep = _Keep()
    obs = keep.arr(np.asarray(obs, dtype=np.float64).reshape(-1, 2), np.float64)
    n_obs = obs.shape[0]
    Np = int(n_particles)
    pay = np.zeros((n_obs, Np))
    tau = np.zeros((n_obs, Np), dtype=np.int64)
    cap = np.zeros((n_obs, Np), dtype=np.uint8)
    ex = np.zeros((n_obs, Np, 2))
    fl = _flow(keep, domain, modes, u, v0)
    ff = _field(keep, f)
    gg = _field(keep, g)
    lib().orc_observe_dirichlet(C.byref(fl), C.byref(ff), C.byref(gg), _ptr(obs, C.c_double),
                                n_obs, kappa, dt, Np, C.c_uint64(int(seed)), int(max_steps),
                                _ptr(pay, C.c_double), _ptr(tau, C.c_int64),
                                _ptr(cap, C.c_uint8), _ptr(ex, C.c_double))
    return {"payoff": pay, "tau_steps": tau, "capped": cap.astype(bool), "exit": ex}


def mean_var(x: np.ndarray, axis: int = -1):
    """Sample mean and unbiased sample variance (the last line of Algorithms 1-2)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[axis]
    m = x.sum(axis=axis) / n
    d = x - np.expand_dims(m, axis)
    v = (d * d).sum(axis=axis) / max(n - 1, 1)
    return m, v


def observe_time(modes, u, theta0, obs, kappa, T, dt, n_particles, seed, v0=(0.0, 0.0)):
    """G_j(u) of Algorithm 1: (mean, var) per observation."""
    pay = observe_time_payoffs(modes, u, theta0, obs, kappa, T, dt, n_particles, seed, v0)
    return mean_var(pay)


def observe_dirichlet(modes, u, f, g, obs, kappa, dt, n_particles, seed, max_steps,
                      v0=(0.0, 0.0), domain="disk"):
    """G_j(u) of Algorithm 2: mean/var of the payoff and of the exit time."""
    r = observe_dirichlet_paths(modes, u, f, g, obs, kappa, dt, n_particles, seed, max_steps, v0, domain)
    m, v = mean_var(r["payoff"])
    tm, tv = mean_var(r["tau_steps"].astype(np.float64) * dt)
    return {"mean": m, "var": v, "tau_mean": tm, "tau_var": tv,
            "n_capped": r["capped"].sum(axis=1)}


def observe_dirichlet_sources(modes, u, g, obs, kappa, dt, n_particles, seed, max_steps, sources,
                              v0=(0.0, 0.0), domain="square"):
    """Theorem 3.2 with a source f = sum_j f_j phi_j, phi_j(x) = exp(-w_j |x - c_j|^2):
    theta(x_i) = E[theta_dD(X_tau)] - sum_j f_j E[int_0^tau phi_j(X_t) dt], so on common
    random numbers G(F) = a - B F exactly.  a (with its variance) comes from a run with
    f = 0, column j of B from a run with g = 0 and f = phi_j (payoff -int phi_j).
    sources: [(cx, cy, w), ...].  Returns (a_mean, a_var, B [n_obs, n_src], tau_mean)."""
    r0 = observe_dirichlet(modes, u, {"kind": "zero", "params": []}, g, obs, kappa, dt, n_particles, seed,
                           max_steps, v0, domain)
    cols = []
    for cx, cy, w in sources:
        rj = observe_dirichlet(modes, u, {"kind": "gauss", "params": [cx, cy, w, 1.0]},
                               {"kind": "zero", "params": []}, obs, kappa, dt, n_particles, seed, max_steps,
                               v0, domain)
        cols.append(-rj["mean"])
    return r0["mean"], r0["var"], np.stack(cols, axis=1), r0["tau_mean"]


def num_threads() -> int:
    return int(lib().orc_num_threads())
