"""MI355X (gfx950) particle forward maps for sparse-observation inverse problems.

Thin ctypes binding of libpm.so (C ABI in include/pm.h).  Every step of the
path runs in the library's HIP kernels; this module only marshals arguments:
torch CUDA tensors provide device memory and the current HIP stream.

The library must be built in-tree first (``python -m paper_1808_10580_amd.build``
or ``__graft_entry__.build()``); importing a function that needs it raises if
libpm.so is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpm.so")

PM_OK, PM_EINVAL, PM_ENOMEM, PM_EDEVICE, PM_ENONFINITE, PM_ECAPPED, PM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
TORUS, DISK, SQUARE = 0, 1, 2
FP32, FP64 = 0, 1
FIELD_KINDS = {"zero": 0, "const": 1, "sinsin": 2, "fourier": 3, "gauss_periodic": 4,
               "cos_m_theta": 5, "exp_linear": 6, "linear": 7, "gauss": 8, "cos_axes": 9}
MAX_SOURCES = 4
NOALLOC_MAX_CHUNKS = 81920  # pm_observe_time_noalloc: n_obs * ceil(Np / 64) at most
MAX_K = 8
MAX_K_MX = 8  # FP32 torus problems with 1 <= K <= MAX_K_MX use the matrix cores by default
MAX_K_DISK_MX = 4  # the same for FP32 disk problems
ENGINES = {"auto": 0, "valu": 1, "mfma": 2}


class PMError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _lib().pm_strerror(status).decode() if _LIBH is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


_LIBH = None
_LIVE_PROBLEMS = weakref.WeakSet()
_LIVE_CONTEXTS = weakref.WeakSet()


@atexit.register
def release_all():
    """Destroy every live library object (graphs, problems, then contexts)."""
    for c in list(_LIVE_CONTEXTS):
        for g in list(getattr(c, "_graphs", ())):
            g.close()
        for m in list(getattr(c, "_mlps", ())):
            m.close()
    for p in list(_LIVE_PROBLEMS):
        p.close()
    for c in list(_LIVE_CONTEXTS):
        c.close()


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_params", C.c_int32), ("params", C.POINTER(C.c_double))]


_vp = C.c_void_p
_d = C.c_double
_i64 = C.c_int64
_u64 = C.c_uint64


def _declare(L):
    L.pm_strerror.restype = C.c_char_p
    L.pm_strerror.argtypes = [C.c_int]
    L.pm_create.argtypes = [C.POINTER(_vp), C.c_int, _vp]
    L.pm_destroy.argtypes = [_vp]
    L.pm_destroy.restype = None
    L.pm_set_stream.argtypes = [_vp, _vp]
    L.pm_set_tuning.argtypes = [_vp, C.c_int, C.c_int]
    L.pm_set_velocity_engine.argtypes = [_vp, C.c_int]
    L.pm_problem_create.argtypes = [_vp, C.POINTER(_vp), C.c_int, C.c_int, _vp, _vp,
                                    C.POINTER(_Field), C.c_int]
    L.pm_problem_destroy.argtypes = [_vp]
    L.pm_problem_destroy.restype = None
    L.pm_observe_time.argtypes = [_vp, _vp, _vp, _vp, C.c_int, _d, _d, _d, _i64, _u64, _vp, _vp, _vp]
    L.pm_observe_time_noalloc.argtypes = [_vp, _vp, _vp, _vp, C.c_int, _d, _d, _d, _i64, _u64, _vp, _vp, _vp]
    L.pm_observe_time_multi.argtypes = [_vp, _vp, _vp, _vp, C.c_int, _vp, C.c_int, _d, _d, _i64, _u64,
                                        _vp, _vp]
    L.pm_jacobian_time.argtypes = [_vp, _vp, _vp, _vp, C.c_int, _d, _d, _d, _i64, _u64, _d, _vp]
    L.pm_replay_path.argtypes = [_vp, _vp, _vp, _vp, C.c_int, _d, _d, _d, _i64, _u64, C.c_int, _i64, _vp]
    L.pm_observe_dirichlet_sources.argtypes = [_vp, _vp, _vp, C.POINTER(_Field), _vp, C.c_int, _d, _d, _i64,
                                               _u64, _i64, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.pm_observe_time_batch.argtypes = [_vp, _vp, C.c_int, _vp, _vp, _vp, _vp, C.c_int, _d, _d, _d,
                                        _vp, _vp]
    L.pm_observe_dirichlet.argtypes = [_vp, _vp, _vp, C.POINTER(_Field), C.POINTER(_Field), _vp,
                                       C.c_int, _d, _d, _i64, _u64, _i64, _vp, _vp, _vp, _vp, _vp, _vp]
    L.pm_step.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _d, _d, _u64, _vp]
    L.pm_velocity.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp]
    L.pm_normals.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp, _u64, _vp]
    L.pm_sync.argtypes = [_vp]
    L.pm_last_kernel_stats.argtypes = [_vp, C.POINTER(_d), C.POINTER(_d)]
    L.pm_set_blocks_per_cu.argtypes = [_vp, C.c_int]
    L.pm_set_dirichlet_source.argtypes = [_vp, C.c_int]
    L.pm_set_dirichlet_blocks_per_cu.argtypes = [_vp, C.c_int]
    L.pm_set_dirichlet_compaction.argtypes = [_vp, C.c_int, C.c_int]
    L.pm_set_dirichlet_tail.argtypes = [_vp, C.c_int, _i64]
    L.pm_dirichlet_tail_walkers.argtypes = [_vp, C.POINTER(_i64)]
    L.pm_autotune_time.argtypes = [_vp, _vp, _vp, _vp, C.c_int, _d, _d, _i64, _u64, C.c_int,
                                   C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(_d)]
    L.pm_graph_create_time.argtypes = [_vp, _vp, C.c_int, _vp, _vp, _vp, _vp, C.c_int, _d, _d, _d,
                                       _vp, _vp, C.POINTER(_vp)]
    L.pm_graph_launch.argtypes = [_vp]
    L.pm_graph_particle_steps.argtypes = [_vp, C.POINTER(_d)]
    L.pm_graph_destroy.argtypes = [_vp]
    L.pm_graph_destroy.restype = None
    L.pm_mlp_create.argtypes = [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _u64, C.POINTER(_vp)]
    L.pm_mlp_destroy.argtypes = [_vp]
    L.pm_mlp_destroy.restype = None
    L.pm_mlp_n_params.argtypes = [_vp]
    L.pm_mlp_n_params.restype = C.c_int64
    L.pm_mlp_set_params.argtypes = [_vp, _vp]
    L.pm_mlp_get_params.argtypes = [_vp, _vp]
    L.pm_mlp_set_io.argtypes = [_vp, _vp, _vp, _vp]
    L.pm_mlp_forward.argtypes = [_vp, _vp, C.c_int, _vp]
    L.pm_mlp_train_step.argtypes = [_vp, _vp, _vp, C.c_int, C.c_float, _vp]
    L.pm_mlp_grads.argtypes = [_vp, _vp, _vp, C.c_int, _vp]
    return L


def _lib():
    global _LIBH
    if _LIBH is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1808_10580_amd.build`")
        _LIBH = _declare(C.CDLL(LIB_PATH))
    return _LIBH


def lib():
    """The loaded libpm.so (ctypes handle)."""
    return _lib()


def _check(st: int, what: str):
    if st != PM_OK:
        raise PMError(st, what)


def _torch():
    import torch
    return torch


def _dev(x, dtype, device):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(np.array(x), dtype=dtype, device=device)
    return t.contiguous()


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class _FieldHolder:
    def __init__(self, fd: Optional[dict]):
        if fd is None:
            fd = {"kind": "zero", "params": []}
        p = np.ascontiguousarray(np.asarray(fd.get("params", []), dtype=np.float64).reshape(-1))
        self.p = p if p.size else np.zeros(1)
        self.s = _Field(FIELD_KINDS[fd["kind"]], int(p.size),
                        self.p.ctypes.data_as(C.POINTER(C.c_double)))


class Context:
    """A libpm context bound to a HIP device; calls enqueue on torch's current stream."""

    def __init__(self, device: int = 0):
        torch = _torch()
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        st = _lib().pm_create(C.byref(h), device, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
        _check(st, "pm_create")
        self.h = h
        self._problems = weakref.WeakSet()
        self._graphs = weakref.WeakSet()
        self._mlps = weakref.WeakSet()
        _LIVE_CONTEXTS.add(self)

    def bind_stream(self):
        torch = _torch()
        _lib().pm_set_stream(self.h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def set_tuning(self, particles_per_lane: int = 0, coef_source: int = 0):
        _check(_lib().pm_set_tuning(self.h, particles_per_lane, coef_source), "pm_set_tuning")

    def set_velocity_engine(self, engine="auto"):
        """Velocity engine of FP32 problems: "auto"/"mfma" (matrix cores for
        torus 1 <= K <= 8 and disk 1 <= K <= 4) or "valu" (vector FMAs; the
        kernel that set_tuning and autotune_time tune)."""
        code = ENGINES[engine] if isinstance(engine, str) else int(engine)
        _check(_lib().pm_set_velocity_engine(self.h, code), "pm_set_velocity_engine")

    def set_dirichlet_source(self, coef_source: int = 1):
        _check(_lib().pm_set_dirichlet_source(self.h, coef_source), "pm_set_dirichlet_source")

    def set_dirichlet_blocks_per_cu(self, blocks_per_cu: int = 0):
        _check(_lib().pm_set_dirichlet_blocks_per_cu(self.h, blocks_per_cu), "pm_set_dirichlet_blocks_per_cu")

    def set_dirichlet_compaction(self, dump_below: int = 0, launches: int = 8):
        _check(_lib().pm_set_dirichlet_compaction(self.h, dump_below, launches), "pm_set_dirichlet_compaction")

    def set_dirichlet_tail(self, live_below: int = 0, hand_steps: int = 0):
        _check(_lib().pm_set_dirichlet_tail(self.h, live_below, hand_steps), "pm_set_dirichlet_tail")

    def dirichlet_tail_walkers(self) -> int:
        n = _i64(0)
        _check(_lib().pm_dirichlet_tail_walkers(self.h, C.byref(n)), "pm_dirichlet_tail_walkers")
        return int(n.value)

    def set_blocks_per_cu(self, blocks_per_cu: int = 0):
        _check(_lib().pm_set_blocks_per_cu(self.h, blocks_per_cu), "pm_set_blocks_per_cu")

    def sync(self, raise_on_flags: bool = False) -> int:
        st = _lib().pm_sync(self.h)
        if st in (PM_EDEVICE, PM_EINVAL) or (raise_on_flags and st != PM_OK):
            raise PMError(st, "pm_sync")
        return st

    def last_kernel_stats(self):
        ms, steps = C.c_double(), C.c_double()
        _check(_lib().pm_last_kernel_stats(self.h, C.byref(ms), C.byref(steps)), "pm_last_kernel_stats")
        return ms.value, steps.value

    def close(self):
        """Destroy the context; its graphs, surrogates and problems first."""
        if getattr(self, "h", None):
            for g in list(getattr(self, "_graphs", ())):
                g.close()
            for s in list(getattr(self, "_mlps", ())):
                s.close()
            for p in list(getattr(self, "_problems", ())):
                p.close()
            _lib().pm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """Problem handle: domain, wavevector table, constant drift, theta0, precision."""

    def __init__(self, ctx: Context, domain: str, modes, v0=(0.0, 0.0), theta0: Optional[dict] = None,
                 prec: str = "fp32"):
        self.ctx = ctx
        self.modes = np.ascontiguousarray(np.asarray(modes, dtype=np.int32).reshape(-1, 2))
        self.n_modes = int(self.modes.shape[0])
        self.domain = domain
        self.prec = prec
        v0a = np.ascontiguousarray(np.asarray(v0, dtype=np.float64).reshape(2))
        th = _FieldHolder(theta0) if theta0 is not None else None
        h = C.c_void_p()
        st = _lib().pm_problem_create(
            ctx.h, C.byref(h), {"torus": TORUS, "disk": DISK, "square": SQUARE}[domain], self.n_modes,
            C.c_void_p(self.modes.ctypes.data) if self.n_modes else None, C.c_void_p(v0a.ctypes.data),
            C.byref(th.s) if th is not None else None, {"fp32": FP32, "fp64": FP64}[prec])
        _check(st, "pm_problem_create")
        self.h = h
        self._graphs = weakref.WeakSet()
        ctx._problems.add(self)
        _LIVE_PROBLEMS.add(self)

    def close(self):
        if getattr(self, "h", None):
            for g in list(getattr(self, "_graphs", ())):
                g.close()
            _lib().pm_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _u(self, u):
        torch = _torch()
        t = _dev(u, torch.float64, self.ctx.device)
        return t

    # -- Algorithm 1 -----------------------------------------------------------------
    def observe_time(self, u, obs, kappa, T, dt, n_particles, seed, endpoints=False):
        """G_j(u) of Algorithm 1: (mean, var[, endpoints]) as CUDA float64 tensors."""
        torch = _torch()
        self.ctx.bind_stream()
        ut = self._u(u)
        ob = _dev(obs, torch.float64, self.ctx.device).reshape(-1, 2)
        n_obs = ob.shape[0]
        mean = torch.empty(n_obs, dtype=torch.float64, device=self.ctx.device)
        var = torch.empty_like(mean)
        ep = (torch.empty((n_obs, int(n_particles), 2), dtype=torch.float64, device=self.ctx.device)
              if endpoints else None)
        st = _lib().pm_observe_time(self.ctx.h, self.h, _ptr(ut), _ptr(ob), n_obs, float(kappa), float(T),
                                    float(dt), int(n_particles), int(seed), _ptr(mean), _ptr(var), _ptr(ep))
        _check(st, "pm_observe_time")
        return (mean, var, ep) if endpoints else (mean, var)

    def observe_time_noalloc(self, u, obs, kappa, T, dt, n_particles, seed, mean, var, endpoints=None):
        """pm_observe_time_noalloc: Algorithm 1 into caller-provided CUDA float64
        tensors mean, var ([n_obs]) and optional endpoints ([n_obs][Np][2]);
        the library allocates no device memory during the call."""
        torch = _torch()
        self.ctx.bind_stream()
        ut = self._u(u)
        ob = _dev(obs, torch.float64, self.ctx.device).reshape(-1, 2)
        n_obs = ob.shape[0]
        for name, t, shape in (("mean", mean, (n_obs,)), ("var", var, (n_obs,)),
                               ("endpoints", endpoints, (n_obs, int(n_particles), 2))):
            if t is None and name == "endpoints":
                continue
            if (t is None or t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != shape
                    or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous CUDA float64 tensor of shape {shape}")
        st = _lib().pm_observe_time_noalloc(self.ctx.h, self.h, _ptr(ut), _ptr(ob), n_obs, float(kappa), float(T),
                                            float(dt), int(n_particles), int(seed), _ptr(mean), _ptr(var),
                                            _ptr(endpoints))
        _check(st, "pm_observe_time_noalloc")
        return mean, var

    def observe_time_multi(self, u, obs, kappa, read_steps: Sequence[int], dt, n_particles, seed):
        """Observations at t_k = read_steps[k] * dt along one ensemble per point:
        (mean, var) as CUDA float64 tensors [n_read, n_obs]."""
        torch = _torch()
        self.ctx.bind_stream()
        ut = self._u(u)
        ob = _dev(obs, torch.float64, self.ctx.device).reshape(-1, 2)
        n_obs = ob.shape[0]
        rs = np.ascontiguousarray(np.asarray(read_steps, dtype=np.int64).reshape(-1))
        mean = torch.empty((rs.size, n_obs), dtype=torch.float64, device=self.ctx.device)
        var = torch.empty_like(mean)
        st = _lib().pm_observe_time_multi(self.ctx.h, self.h, _ptr(ut), _ptr(ob), n_obs, C.c_void_p(rs.ctypes.data),
                                          int(rs.size), float(kappa), float(dt), int(n_particles), int(seed),
                                          _ptr(mean), _ptr(var))
        _check(st, "pm_observe_time_multi")
        return mean, var

    def replay_path(self, u, obs, kappa, T, dt, n_particles, seed, j, i):
        """Positions X_0..X_{N_t} of particle i of observation j in the map
        observe_time(u, obs, kappa, T, dt, n_particles, seed): a CUDA float64
        tensor [N_t + 1, 2], wrapped to [0,1)^2."""
        torch = _torch()
        self.ctx.bind_stream()
        ut = self._u(u)
        ob = _dev(obs, torch.float64, self.ctx.device).reshape(-1, 2)
        nt = n_steps(float(T), float(dt))
        path = torch.empty((nt + 1, 2), dtype=torch.float64, device=self.ctx.device)
        st = _lib().pm_replay_path(self.ctx.h, self.h, _ptr(ut), _ptr(ob), ob.shape[0], float(kappa), float(T),
                                   float(dt), int(n_particles), int(seed), int(j), int(i), _ptr(path))
        _check(st, "pm_replay_path")
        return path

    def jacobian_time(self, u, obs, kappa, T, dt, n_particles, seed, h):
        """Central-difference Jacobian dG/du [n_obs, 2M] with common random numbers (one batched launch)."""
        torch = _torch()
        self.ctx.bind_stream()
        ut = self._u(u)
        ob = _dev(obs, torch.float64, self.ctx.device).reshape(-1, 2)
        J = torch.empty((ob.shape[0], 2 * self.n_modes), dtype=torch.float64, device=self.ctx.device)
        st = _lib().pm_jacobian_time(self.ctx.h, self.h, _ptr(ut), _ptr(ob), ob.shape[0], float(kappa), float(T),
                                     float(dt), int(n_particles), int(seed), float(h), _ptr(J))
        _check(st, "pm_jacobian_time")
        return J

    def observe_time_batch(self, U, n_particles: Sequence[int], seeds: Sequence[int], obs, kappa, T, dt):
        torch = _torch()
        self.ctx.bind_stream()
        Ut = _dev(U, torch.float64, self.ctx.device).reshape(-1, 2 * self.n_modes if self.n_modes else 0)
        n_u = int(len(n_particles))
        ob = _dev(obs, torch.float64, self.ctx.device).reshape(-1, 2)
        n_obs = ob.shape[0]
        nps = np.ascontiguousarray(np.asarray(n_particles, dtype=np.int64))
        sds = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
        mean = torch.empty((n_u, n_obs), dtype=torch.float64, device=self.ctx.device)
        var = torch.empty_like(mean)
        st = _lib().pm_observe_time_batch(self.ctx.h, self.h, n_u, _ptr(Ut), C.c_void_p(nps.ctypes.data),
                                          C.c_void_p(sds.ctypes.data), _ptr(ob), n_obs, float(kappa),
                                          float(T), float(dt), _ptr(mean), _ptr(var))
        _check(st, "pm_observe_time_batch")
        return mean, var

    def autotune_time(self, u, obs, kappa, dt, n_particles, seed=1, n_probe_steps=100):
        """Time every variant of the kernel this problem runs on (vector engine:
        particles per lane and coefficient source; matrix-core engine: blocks
        per compute unit) on a probe and keep the fastest for this K."""
        torch = _torch()
        self.ctx.bind_stream()
        ut = self._u(u)
        ob = _dev(obs, torch.float64, self.ctx.device).reshape(-1, 2)
        ppl, src, bpc, ms = C.c_int(), C.c_int(), C.c_int(), C.c_double()
        st = _lib().pm_autotune_time(self.ctx.h, self.h, _ptr(ut), _ptr(ob), ob.shape[0], float(kappa),
                                     float(dt), int(n_particles), int(seed), int(n_probe_steps),
                                     C.byref(ppl), C.byref(src), C.byref(bpc), C.byref(ms))
        _check(st, "pm_autotune_time")
        return {"particles_per_lane": ppl.value, "coef_source": src.value, "blocks_per_cu": bpc.value,
                "probe_ms": ms.value}

    def graph_time(self, u, obs, kappa, T, dt, n_particles, seeds) -> "Graph":
        """Capture pm_observe_time_batch (n_u = len(n_particles)) as a replayable graph.
        ``u`` and ``obs`` must be CUDA float64 tensors the caller keeps and updates
        in place between replays; the graph's outputs are ``graph.mean``/``graph.var``."""
        return Graph(self, u, obs, kappa, T, dt, n_particles, seeds)

    # -- Algorithm 2 -----------------------------------------------------------------
    def observe_dirichlet(self, u, f: dict, g: dict, obs, kappa, dt, n_particles, seed, max_steps,
                          paths=False):
        torch = _torch()
        self.ctx.bind_stream()
        ut = self._u(u)
        ob = _dev(obs, torch.float64, self.ctx.device).reshape(-1, 2)
        n_obs = ob.shape[0]
        dev = self.ctx.device
        out = {k: torch.empty(n_obs, dtype=torch.float64, device=dev)
               for k in ("mean", "var", "tau_mean", "tau_var")}
        out["n_capped"] = torch.empty(n_obs, dtype=torch.int64, device=dev)
        pt = (torch.empty((n_obs, int(n_particles), 4), dtype=torch.float64, device=dev) if paths else None)
        ff, gg = _FieldHolder(f), _FieldHolder(g)
        st = _lib().pm_observe_dirichlet(self.ctx.h, self.h, _ptr(ut), C.byref(ff.s), C.byref(gg.s), _ptr(ob),
                                         n_obs, float(kappa), float(dt), int(n_particles), int(seed),
                                         int(max_steps), _ptr(out["mean"]), _ptr(out["var"]),
                                         _ptr(out["tau_mean"]), _ptr(out["tau_var"]), _ptr(out["n_capped"]),
                                         _ptr(pt))
        _check(st, "pm_observe_dirichlet")
        if paths:
            out["paths"] = pt
        return out

    def observe_dirichlet_sources(self, u, g: dict, obs, kappa, dt, n_particles, seed, max_steps, sources):
        """Theorem 3.2 split by Gaussian sources (PM_SQUARE): a = E[theta_dD(X_tau)] and
        B[q, i] = E[int phi_q(X_t) dt], so G(F) = a - B^T F.  sources: [(cx, cy, w), ...]."""
        torch = _torch()
        self.ctx.bind_stream()
        ut = self._u(u)
        ob = _dev(obs, torch.float64, self.ctx.device).reshape(-1, 2)
        n_obs = ob.shape[0]
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.float64).reshape(-1, 3))
        dev = self.ctx.device
        out = {k: torch.empty(n_obs, dtype=torch.float64, device=dev)
               for k in ("bnd_mean", "bnd_var", "tau_mean", "tau_var")}
        out["B"] = torch.empty((src.shape[0], n_obs), dtype=torch.float64, device=dev)
        out["n_capped"] = torch.empty(n_obs, dtype=torch.int64, device=dev)
        gg = _FieldHolder(g)
        st = _lib().pm_observe_dirichlet_sources(
            self.ctx.h, self.h, _ptr(ut), C.byref(gg.s), _ptr(ob), n_obs, float(kappa), float(dt),
            int(n_particles), int(seed), int(max_steps), int(src.shape[0]), C.c_void_p(src.ctypes.data),
            _ptr(out["bnd_mean"]), _ptr(out["bnd_var"]), _ptr(out["B"]), _ptr(out["tau_mean"]),
            _ptr(out["tau_var"]), _ptr(out["n_capped"]))
        _check(st, "pm_observe_dirichlet_sources")
        return out

    # -- replay / inspection ---------------------------------------------------------
    def step(self, u, X, n, i, j, kappa, dt, seed):
        torch = _torch()
        self.ctx.bind_stream()
        dev = self.ctx.device
        Xt = _dev(X, torch.float64, dev).reshape(-1, 2)
        cnt = Xt.shape[0]
        nt = _dev(np.broadcast_to(np.asarray(n, dtype=np.int64), (cnt,)), torch.int64, dev)
        it = _dev(np.broadcast_to(np.asarray(i, dtype=np.int64), (cnt,)).astype(np.int32), torch.int32, dev)
        jt = _dev(np.broadcast_to(np.asarray(j, dtype=np.int64), (cnt,)).astype(np.int32), torch.int32, dev)
        Y = torch.empty_like(Xt)
        st = _lib().pm_step(self.ctx.h, self.h, _ptr(self._u(u)), cnt, _ptr(Xt), _ptr(nt), _ptr(it), _ptr(jt),
                            float(kappa), float(dt), int(seed), _ptr(Y))
        _check(st, "pm_step")
        return Y

    def velocity(self, u, X):
        torch = _torch()
        self.ctx.bind_stream()
        Xt = _dev(X, torch.float64, self.ctx.device).reshape(-1, 2)
        V = torch.empty_like(Xt)
        st = _lib().pm_velocity(self.ctx.h, self.h, _ptr(self._u(u)), Xt.shape[0], _ptr(Xt), _ptr(V))
        _check(st, "pm_velocity")
        return V

    def normals(self, n, i, j, seed):
        torch = _torch()
        self.ctx.bind_stream()
        dev = self.ctx.device
        n = np.atleast_1d(np.asarray(n, dtype=np.int64))
        cnt = n.size
        nt = _dev(n, torch.int64, dev)
        it = _dev(np.broadcast_to(np.asarray(i, dtype=np.int64), (cnt,)).astype(np.int32), torch.int32, dev)
        jt = _dev(np.broadcast_to(np.asarray(j, dtype=np.int64), (cnt,)).astype(np.int32), torch.int32, dev)
        Z = torch.empty((cnt, 2), dtype=torch.float64, device=dev)
        st = _lib().pm_normals(self.ctx.h, self.h, cnt, _ptr(nt), _ptr(it), _ptr(jt), int(seed), _ptr(Z))
        _check(st, "pm_normals")
        return Z


class Graph:
    """A captured forward map (pm_graph_create_time); replay() re-reads u and obs."""

    def __init__(self, prob: Problem, u, obs, kappa, T, dt, n_particles, seeds):
        torch = _torch()
        ctx = prob.ctx
        ctx.bind_stream()
        if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()):
            raise TypeError("u must be a contiguous CUDA float64 tensor kept alive by the caller")
        if not (isinstance(obs, torch.Tensor) and obs.is_cuda and obs.dtype == torch.float64 and obs.is_contiguous()):
            raise TypeError("obs must be a contiguous CUDA float64 tensor kept alive by the caller")
        nps = np.ascontiguousarray(np.atleast_1d(np.asarray(n_particles, dtype=np.int64)))
        sds = np.ascontiguousarray(np.atleast_1d(np.asarray(seeds, dtype=np.uint64)))
        n_u = int(nps.size)
        n_obs = obs.numel() // 2
        self.u, self.obs = u, obs
        shape = (n_u, n_obs) if n_u > 1 else (n_obs,)
        self.mean = torch.empty(shape, dtype=torch.float64, device=ctx.device)
        self.var = torch.empty_like(self.mean)
        h = C.c_void_p()
        st = _lib().pm_graph_create_time(ctx.h, prob.h, n_u, _ptr(u), C.c_void_p(nps.ctypes.data),
                                         C.c_void_p(sds.ctypes.data), _ptr(obs), n_obs, float(kappa),
                                         float(T), float(dt), _ptr(self.mean), _ptr(self.var), C.byref(h))
        _check(st, "pm_graph_create_time")
        self.h = h
        self.ctx = ctx
        self.prob = prob
        ctx._graphs.add(self)
        prob._graphs.add(self)

    def replay(self):
        self.ctx.bind_stream()
        _check(_lib().pm_graph_launch(self.h), "pm_graph_launch")
        return self.mean, self.var

    def particle_steps(self) -> float:
        s = C.c_double()
        _check(_lib().pm_graph_particle_steps(self.h, C.byref(s)), "pm_graph_particle_steps")
        return s.value

    def close(self):
        if getattr(self, "h", None):
            _lib().pm_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """Surrogate MLP on the GPU (include/pm_mlp.h): BF16 MFMA GEMMs with FP32
    accumulation, FP32 master weights and Adam."""

    def __init__(self, ctx: Context, d_in: int, d_hidden: int, n_hidden: int, d_out: int, max_batch: int,
                 seed: int = 0):
        h = C.c_void_p()
        _check(_lib().pm_mlp_create(ctx.h, d_in, d_hidden, n_hidden, d_out, max_batch, int(seed), C.byref(h)),
               "pm_mlp_create")
        self.h, self.ctx = h, ctx
        self.dims = (d_in, d_hidden, n_hidden, d_out)
        self.max_batch = max_batch
        self.n_params = int(_lib().pm_mlp_n_params(h))
        torch = _torch()
        self._loss = torch.zeros(1, dtype=torch.float32, device=ctx.device)
        ctx._mlps.add(self)

    def _f32(self, x):
        torch = _torch()
        return _dev(x, torch.float32, self.ctx.device)

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        assert p.size == self.n_params
        _check(_lib().pm_mlp_set_params(self.h, C.c_void_p(p.ctypes.data)), "pm_mlp_set_params")

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.n_params, dtype=np.float32)
        _check(_lib().pm_mlp_get_params(self.h, C.c_void_p(p.ctypes.data)), "pm_mlp_get_params")
        return p

    def set_io(self, in_scale=None, out_mean=None, out_std=None):
        arrs = [None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float32))
                for a in (in_scale, out_mean, out_std)]
        ptrs = [None if a is None else C.c_void_p(a.ctypes.data) for a in arrs]
        _check(_lib().pm_mlp_set_io(self.h, *ptrs), "pm_mlp_set_io")

    def forward(self, x):
        torch = _torch()
        self.ctx.bind_stream()
        xt = self._f32(x).reshape(-1, self.dims[0])
        y = torch.empty((xt.shape[0], self.dims[3]), dtype=torch.float32, device=self.ctx.device)
        _check(_lib().pm_mlp_forward(self.h, _ptr(xt), xt.shape[0], _ptr(y)), "pm_mlp_forward")
        return y

    def train_step(self, x, t, lr: float):
        self.ctx.bind_stream()
        xt = self._f32(x).reshape(-1, self.dims[0])
        tt = self._f32(t).reshape(-1, self.dims[3])
        _check(_lib().pm_mlp_train_step(self.h, _ptr(xt), _ptr(tt), xt.shape[0], float(lr), _ptr(self._loss)),
               "pm_mlp_train_step")
        return self._loss

    def grads(self, x, t) -> np.ndarray:
        self.ctx.bind_stream()
        xt = self._f32(x).reshape(-1, self.dims[0])
        tt = self._f32(t).reshape(-1, self.dims[3])
        g = np.zeros(self.n_params, dtype=np.float32)
        _check(_lib().pm_mlp_grads(self.h, _ptr(xt), _ptr(tt), xt.shape[0], C.c_void_p(g.ctypes.data)),
               "pm_mlp_grads")
        return g

    def close(self):
        if getattr(self, "h", None):
            _lib().pm_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def n_steps(T: float, dt: float) -> int:
    """Number of uniform steps the library takes to reach T: ceil(T/dt) (to 1e-9)."""
    import math
    return int(math.ceil(T / dt - 1e-9))
