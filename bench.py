#!/usr/bin/env python3
"""Throughput of the particle forward map on one MI355X.

One benchmark step is one evaluation of G(u) (Algorithm 1) on the main torus
workload: 49 observation points on a 7x7 grid, 1e5 particles each, 1000
Euler-Maruyama steps (T = 1, dt = 1e-3), a stream function with 168 Fourier
coefficients (|k|_inf <= 6), FP32 particle states with FP64 payoffs and
statistics -- 4.9e9 particle-steps per step.  Inputs are seeded synthetic
draws; u and the observation points are resident in HBM before timing, and
each step ends when the 49 means are back on the host (as an MCMC step needs).

Prints one JSON line:
  value            particle-steps/s over the K timed steps (wall clock)
  roofline         the time kernel's rate in algorithmic FLOPs -- the
                   mode-by-mode sum of eq. v_expand, 14 FLOP per mode, 12 per
                   harmonic, 20 for the update and the normals -- from HIP
                   events on its stream, against the peak of the unit that
                   runs the velocity contraction (the dense FP16 matrix peak
                   for the default matrix-core engine, the FP32 vector peak
                   for the vector engine); beside it the FLOPs the kernel
                   executes and, from rocprofv3 counters, what limits it
  cpu_baseline     the FP64 CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector peak: 256 CU x 2.4 GHz x 256 FLOP/clk/CU

# HBM bytes per launch of the time kernel on this workload, from rocprofv3's
# FETCH_SIZE and WRITE_SIZE counters scaled by what they read for a plain copy
# of known size (the copy kernel reads FETCH_SIZE at 0.5 and WRITE_SIZE at 1.0
# of the bytes moved).  Valid only for the kernel sources they were taken on:
# reported when the sources still hash to the recorded value, else null.
# Per velocity engine: (bytes per launch, SHA-256 of the kernel's sources).
COUNTER_TRAFFIC = {
    # k_time<float,6,3>: FETCH 161.81 KiB x 2 + WRITE 77,480.78 KiB x 1
    "valu": (79_671_711, "900da7bf51e4b4156b12bf2f83a11f1379e33170f399d1018a0315eba7620f49"),
    # k_time_mx<6>: FETCH 60.69 KiB x 2 + WRITE 40,846.84 KiB x 1
    "mfma": (41_951_457, "def84aa17d9394b534620b9ddc860714a7a4d32c75dac12019d9daa3a412b344"),
}
# The same for the dominant kernel of the other workloads (bench.py
# --workload ...), keyed by (workload, velocity engine): (bytes per launch,
# SHA-256 of the sources, source list).
OTHER_TRAFFIC = {
    # k_time_hk<6,2>: FETCH 928.31 KiB x 2 + WRITE 40,702.97 KiB x 1
    ("torus-k80-turbulent", "mfma"): (43_581_023, "6912bad040a8595f18a03950f3a6507e174bee024c5640f766a4fd3b522fee09", "hk"),
    # k_dirichlet_mx<4,0> (the map's first launch; the cooperative tail adds FETCH 1,346 KiB x 2 +
    # WRITE 1,152 KiB): FETCH 71.38 KiB x 2 + WRITE 80,384.97 KiB x 1
    ("disk-dirichlet", "mfma"): (82_460_384, "1139ace9298341cf2fb91a61b92203356194799916f171e6fb5854069a02bcfd", "mfma_disk"),
    # k_dirichlet<float,4,0,SC>: FETCH 137.94 KiB x 2 + WRITE 80,194.91 KiB x 1
    ("disk-dirichlet", "valu"): (82_402_081, "900da7bf51e4b4156b12bf2f83a11f1379e33170f399d1018a0315eba7620f49", "valu"),
}
KERNEL_SOURCES = {
    "hk": ("paper_1808_10580_amd/csrc/pm_device.h", "paper_1808_10580_amd/csrc/pm_kernels.h",
           "paper_1808_10580_amd/csrc/pm_split.h", "paper_1808_10580_amd/csrc/pm_hk.hip"),
    "valu": ("paper_1808_10580_amd/csrc/pm_device.h", "paper_1808_10580_amd/csrc/pm_kernels.h",
             "paper_1808_10580_amd/csrc/pm_walk.h", "paper_1808_10580_amd/csrc/pm_kernels.hip"),
    "mfma": ("paper_1808_10580_amd/csrc/pm_device.h", "paper_1808_10580_amd/csrc/pm_kernels.h",
             "paper_1808_10580_amd/csrc/pm_walk.h", "paper_1808_10580_amd/csrc/pm_mx.h",
             "paper_1808_10580_amd/csrc/pm_split.h", "paper_1808_10580_amd/csrc/pm_mx.hip"),
    # the disk walk's traffic also depends on the host side's launch settings
    # (the tail's hand-over threshold, blocks per compute unit)
    "mfma_disk": ("paper_1808_10580_amd/csrc/pm_device.h", "paper_1808_10580_amd/csrc/pm_kernels.h",
                  "paper_1808_10580_amd/csrc/pm_walk.h", "paper_1808_10580_amd/csrc/pm_mx.h",
                  "paper_1808_10580_amd/csrc/pm_split.h", "paper_1808_10580_amd/csrc/pm_mx.hip",
                  "paper_1808_10580_amd/csrc/pm_abi.hip"),
}
# Matrix-core FLOPs issued per particle-step by the small-K engine: per 64
# particles two 32-column blocks x three v_mfma_f32_32x32x16_f16 (32 x 32 x 16
# multiply-adds each), padding included.
MX_ISSUED_FLOP_PER_PARTICLE_STEP = 2 * 3 * 2 * 32 * 32 * 16 // 64
PEAK_FP16_DENSE_TFLOPS = 2500.0

# rocprofv3 counters of the time kernel on the main workload (per particle-step:
# counter x 64 lanes / 4.9e9), valid for the sources they were taken on.
# Keys: VALU instructions, VALU issue slots (multi-cycle operations count their
# extra cycles), FP32 FMA / MUL / ADD instructions, matrix-core busy fraction,
# and the fraction of the kernel's cycles one VALU issue port needs for the
# slots (slots x 4 cycles per wave64 slot / 64 lanes per wave, over the
# kernel's cycles per SIMD).
COUNTERS = {
    "mfma": ({"valu_insts": 130.1, "valu_slots": 164.1, "fma_f32": 47.0, "mul_f32": 6.0, "add_f32": 4.0,
              "issue_frac": 1.03, "mfma_busy": 0.301,
              "source": "profiles/k_time_mx_torus-k6-fp32_pmc.md"},
             "def84aa17d9394b534620b9ddc860714a7a4d32c75dac12019d9daa3a412b344"),
    "valu": (None, ""),
}


def kernel_sources_sha256(engine: str = "valu") -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[engine]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(engine: str):
    nbytes, sha = COUNTER_TRAFFIC[engine]
    if nbytes is None or kernel_sources_sha256(engine) != sha:
        return None
    return nbytes


def other_traffic(workload: str, engine: str):
    nbytes, sha, src = OTHER_TRAFFIC.get((workload, engine), (None, "", "valu"))
    if nbytes is None or kernel_sources_sha256(src) != sha:
        return None
    return nbytes


def calibration_copy(torch, dev, mib: int):
    """One plain device-to-device copy of a known size: the reference that
    scales the profiler's FETCH_SIZE / WRITE_SIZE counters to bytes."""
    if mib > 0:
        src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst


def engine_in_use(pm, engine_arg: str, K: int, domain: str = "torus") -> str:
    """The velocity engine the library runs for an FP32 torus or disk problem."""
    limit = pm.MAX_K_MX if domain == "torus" else pm.MAX_K_DISK_MX
    if engine_arg == "valu" or not (1 <= K <= limit):
        return "valu"
    return "mfma"


def counters(engine: str):
    """The recorded counter figures of the time kernel, or None once its
    sources have changed since they were taken."""
    fig, sha = COUNTERS[engine]
    if fig is None or kernel_sources_sha256(engine) != sha:
        return None
    return fig


def kernel_roofline(engine: str, K: int, fl: int, fl_exec: int, steps: float, kern_s: float, traffic):
    """Roofline of the time kernel.  `fl`: algorithmic FLOPs per particle-step
    (the mode-by-mode sum); `fl_exec`: the FP32-equivalent FLOPs the kernel's
    tensor-product velocity executes.  The bound is the unit that runs the
    velocity contraction: the FP16 matrix cores (split FP16 x3, FP32
    accumulation) for the matrix-core engine, the FP32 vector units otherwise."""
    achieved = fl * steps / kern_s / 1e12
    mx = engine == "mfma"
    peak = PEAK_FP16_DENSE_TFLOPS if mx else PEAK_FP32_TFLOPS
    rl = {"bound": "mfma" if mx else "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
          "frac": round(achieved / peak, 4), "traffic": traffic, "traffic_unit": "bytes per launch",
          "peak_of": "dense FP16 matrix" if mx else "FP32 vector (256 CU x 2.4 GHz x 256 FLOP/clk)",
          "kernel": "k_time_mx<%d>" % K if mx else "k_time<float,%d>" % K,
          "kernel_ms": round(kern_s * 1e3, 3), "flop_per_particle_step": fl,
          "flop_count": "mode sum of eq. v_expand: 14 per mode + 12 per harmonic + 20 (update, normals)",
          "executed_flop_per_particle_step": fl_exec,
          "executed_tflops": round(fl_exec * steps / kern_s / 1e12, 3), "engine": engine}
    if mx:
        issued = MX_ISSUED_FLOP_PER_PARTICLE_STEP * steps / kern_s / 1e12
        rl["matrix_cores"] = {"contraction": "split FP16 x3 (hi*hi + hi*lo + lo*hi), FP32 accumulate",
                              "issued_tflops": round(issued, 2), "frac_issued": round(issued / PEAK_FP16_DENSE_TFLOPS, 4)}
    c = counters(engine)
    if c is not None:
        fp32 = (2 * c["fma_f32"] + c["mul_f32"] + c["add_f32"]) * steps / kern_s / 1e12
        rl["limiter"] = {"unit": "VALU issue", "valu_insts_per_particle_step": c["valu_insts"],
                         "valu_issue_slots_per_particle_step": c["valu_slots"],
                         "one_port_issue_frac": c["issue_frac"], "matrix_core_busy": c.get("mfma_busy"),
                         "counted_fp32_valu_tflops": round(fp32, 2),
                         "counted_fp32_valu_frac": round(fp32 / PEAK_FP32_TFLOPS, 4),
                         "source": c["source"]}
    return rl


def alg_flops_per_particle_step(n_modes: int, K: int, domain: str = "torus") -> int:
    """Algorithmic FLOPs of one Euler-Maruyama step (FMA = 2) by the method's
    own arithmetic, the mode-by-mode sum of eq. v_expand: per mode the
    sine and cosine of 2 pi k.x from the axis values by angle addition
    (6 FLOP) and two FMAs per velocity component (8); per harmonic of each
    axis one angle-addition step (6 FLOP per axis, 12 per harmonic); the
    update and Box-Muller arithmetic 20.  The disk's stream function carries a
    third form (psi itself, for the cutoff's product rule: 4 more per mode)
    and the cutoff (16 more).  The hardware transcendentals and the Philox
    integer work carry no FLOPs."""
    if domain == "disk":
        return 18 * n_modes + 12 * K + 36
    return 14 * n_modes + 12 * K + 20


def flops_per_particle_step(K: int) -> int:
    """FP32-equivalent FLOPs the tensor-product time kernels execute per
    Euler-Maruyama step (FMA = 2).  Trig basis: per axis K-1 three-term
    recurrence harmonics of 2 FMA (4 FLOP) after one sin/cos pair.  Velocity:
    two bilinear forms phi(x)^T C phi(y) over B = 2K+1 basis functions per
    axis; row j = 0 carries only the y form (1 mul + (B-2) FMA), rows j >= 1
    carry both (x: B-1 FMA, y: 1 mul + B-2 FMA) and two FMAs into (v_x, v_y).
    Update: 1 add + 2 FMA per axis.  Box-Muller arithmetic: 1 FMA + 4 mul per
    normal pair.  The 8 hardware transcendentals and the Philox integer work
    are not counted."""
    B = 2 * K + 1
    basis = 2 * (K - 1) * 4
    row0 = 1 + 2 * (B - 2)
    row = 2 * (B - 1) + (1 + 2 * (B - 2)) + 2 * 2
    contraction = row0 + (B - 1) * row
    update = 2 * (1 + 2 * 2)
    bm = 2 + 4
    return basis + contraction + update + bm


def flops_per_particle_step_disk(K: int) -> int:
    """FP32-equivalent FLOPs one step of the Dirichlet walk on the disk executes:
    three bilinear forms (psi_F and its two derivatives) over B = 2K+1 basis
    functions, 3 (B-1) + 3 FMA per row; the trig basis as on the torus; the
    cutoff (1 - r^2)^2 and its product rule (13); the update and Box-Muller
    arithmetic as on the torus.  The FP64 exit test and source sum are not
    counted."""
    B = 2 * K + 1
    basis = 2 * (K - 1) * 4
    contraction = B * (3 * (B - 1) + 3) * 2
    return basis + contraction + 13 + 2 * (1 + 2 * 2) + (2 + 4)


def flops_per_particle_step_mfma(K: int) -> int:
    """Split-FP16 matrix-core FLOPs of one step of the high-wavenumber path:
    two bilinear forms over B = 2K+1 basis functions (2 B^2 multiply-adds) in
    three FP16 products each (hi hi, hi lo, lo hi).  Padding of the tiles to
    32 x 16 is not counted."""
    B = 2 * K + 1
    return 3 * 2 * B * B * 2


def dtype_label(engine: str) -> str:
    """What the velocity contraction computes in: FP16 hi + lo operand pairs,
    three products with FP32 accumulation on the matrix cores, or FP32 FMAs."""
    return "f16x3-split/f32-acc" if engine == "mfma" else "f32"


DTYPE_DETAIL = {
    "mfma": "velocity contraction on the matrix cores in split FP16 (hi*hi + hi*lo + lo*hi, FP32 accumulate); "
            "bases, y form and normals FP32; particle state 32-bit fixed point; payoffs and statistics FP64",
    "valu": "velocity, bases and normals FP32; particle state FP32 hi + lo pair; payoffs and statistics FP64",
}


def cpu_baseline(wl, n_particles: int):
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    oracle.observe_time(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, wl.T, wl.dt, n_particles, wl.seed)
    dt = time.perf_counter() - t0
    steps = wl.n_obs * n_particles * wl.n_steps
    return {"value": steps / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{wl.n_obs} points x {n_particles} particles x {wl.n_steps} steps "
                      f"({steps:.3g} particle-steps, {dt:.1f} s)"}


def _time_steps(run, steps, warmup, ctx):
    import torch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    kernel_ms, work = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
        ms, w = ctx.last_kernel_stats()
        kernel_ms.append(ms)
        work.append(w)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, kernel_ms, work


def bench_modes_sweep(args):
    """Cost of the forward map against the number of modes N_u (the paper's
    cost model is linear in N_u): Euclidean balls |k|_2 <= R of the turbulent
    workload's problem (2 points x 1e5 particles, kappa 3e-5, dt = 1/9600),
    960 steps each, the fastest of three maps per R.  Prints one JSON line with
    a row per R (and the vector engine beside the default for K <= 8)."""
    import numpy as np
    import torch
    import paper_1808_10580_amd as pm
    import workloads as W

    wl = W.turbulent_k80()
    ctx = pm.Context(0)
    obs = torch.tensor(wl.obs, dtype=torch.float64, device="cuda")
    nst = 960
    rows = []
    for R in (4, 6, 8, 12, 16, 24, 32, 40, 48, 64, 80):
        full = W.l2_ball_modes(float(R))
        modes = W.half_plane(full)
        u = torch.tensor(W.draw_prior(modes, np.random.default_rng([W.WORKLOAD_SEED, R])), dtype=torch.float64,
                         device="cuda")
        prob = pm.Problem(ctx, "torus", modes, theta0=wl.theta0, prec="fp32")
        K = int(np.abs(modes).max())
        for eng in (("auto", "valu") if K <= pm.MAX_K else ("auto",)):
            ctx.set_velocity_engine(eng)
            ms = []
            for _ in range(3):
                prob.observe_time(u, obs, wl.kappa, nst * wl.dt, wl.dt, wl.n_particles, wl.seed)
                st = ctx.sync()
                if st != pm.PM_OK:
                    raise pm.PMError(st, "forward map")
                ms.append(ctx.last_kernel_stats()[0])
            steps = 2 * wl.n_particles * nst
            path = ("matrix cores, small K" if engine_in_use(pm, eng, K) == "mfma"
                    else ("vector units" if K <= pm.MAX_K else "matrix cores, high K"))
            rows.append({"R": R, "K": K, "N_u": int(len(full)), "path": path, "kernel_ms": round(min(ms), 3),
                         "ns_per_particle_step": round(min(ms) * 1e6 / steps, 4)})
            print(f"[bench] R={R} N_u={len(full)} {path}: {min(ms):.3f} ms", file=sys.stderr, flush=True)
        ctx.set_velocity_engine("auto")
        prob.close()
    print(json.dumps({"metric": "forward-map time per particle-step against N_u", "unit": "ns",
                      "data": "synthetic", "config": {"workload": "torus-modes-sweep: |k|_2 <= R, 2 points x 1e5 "
                                                                  "particles, 960 steps, kappa 3e-5"},
                      "rows": rows}))
    ctx.close()


def bench_other(args):
    """Secondary workloads (not the default line): the turbulent |k|_2 <= 80
    problem on the matrix cores, the Dirichlet walk on the disk, and the
    512-set batch.  Same JSON keys as the main line."""
    import torch
    import paper_1808_10580_amd as pm
    import workloads as W

    dev = torch.device("cuda", 0)
    ctx = pm.Context(0)
    ctx.set_velocity_engine(args.engine)
    if args.dir_tail >= 0:
        ctx.set_dirichlet_tail(args.dir_tail, args.dir_hand)
    if args.dir_bpc > 0:
        ctx.set_dirichlet_blocks_per_cu(args.dir_bpc)
    name = args.workload
    cpu = None
    calibration_copy(torch, dev, args.copy_mib)
    if name == "torus-k80-turbulent":
        wl = W.turbulent_k80()
        prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
        u = torch.tensor(wl.u, dtype=torch.float64, device=dev)
        obs = torch.tensor(wl.obs, dtype=torch.float64, device=dev)
        reads = wl.extra["read_steps"]

        def run():
            m, _ = prob.observe_time_multi(u, obs, wl.kappa, reads, wl.dt, wl.n_particles, wl.seed)
            m.cpu()
            if ctx.sync() != pm.PM_OK:
                raise pm.PMError(ctx.sync(), "forward map")
        K = int(abs(wl.modes).max())
        fl = alg_flops_per_particle_step(len(wl.modes), K)
        B = 2 * K + 1
        rl = {"bound": "mfma", "peak": PEAK_FP16_DENSE_TFLOPS, "unit": "TFLOP/s",
              "kernel": f"k_time_hk<{(2 * K + 32) // 32}>", "flop_per_particle_step": fl,
              "flop_count": "mode sum of eq. v_expand: 14 per mode + 12 per harmonic + 20 (update, normals)",
              "peak_of": "dense FP16 matrix",
              # the tensor-product contraction, one product per term (2 forms x B^2 multiply-adds)
              "executed_flop_per_particle_step": 2 * B * B * 2,
              # the same with the three split-FP16 products per term
              "issued_flop_per_particle_step": flops_per_particle_step_mfma(K)}
        traffic = other_traffic(name, "mfma")
        desc = ("torus-k80-turbulent: |k|_2<=80 (10,040 modes, 20,080 coefficients), kappa=3e-5, 2 points x 1e5 "
                "particles, 4,800 steps (dt=1/9600) read out at 13 times in [0, 0.5], FP32 states, split-FP16 "
                "matrix-core velocity")
        if not args.no_cpu_baseline:
            import oracle
            oracle.build(force=False)
            n_or, n_st = 256, 400
            t0 = time.perf_counter()
            oracle.observe_time(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, n_st * wl.dt, wl.dt, n_or, wl.seed)
            el = time.perf_counter() - t0
            cpu = {"value": wl.n_obs * n_or * n_st / el, "unit": "particle-steps/s", "cores": oracle.num_threads(),
                   "kind": "oracle", "sample": f"2 points x {n_or} particles x {n_st} steps ({el:.1f} s)"}
    elif name == "disk-dirichlet":
        wl = W.dirichlet_main()
        prob = pm.Problem(ctx, "disk", wl.modes, prec="fp32")
        u = torch.tensor(wl.u, dtype=torch.float64, device=dev)
        obs = torch.tensor(wl.obs, dtype=torch.float64, device=dev)
        last = {}

        def run():
            out = prob.observe_dirichlet(u, wl.f, wl.g, obs, wl.kappa, wl.dt, wl.n_particles, wl.seed, wl.max_steps)
            tau = out["tau_mean"].cpu().numpy()
            out["mean"].cpu()
            st = ctx.sync()
            if st != pm.PM_OK:
                raise pm.PMError(st, "forward map")
            last["steps"] = float((tau / wl.dt).sum() * wl.n_particles)
        K = int(abs(wl.modes).max())
        fl = alg_flops_per_particle_step(len(wl.modes), K, "disk")
        eng = engine_in_use(pm, args.engine, K, "disk")
        mx = eng == "mfma"
        tail_on = mx and (args.dir_tail != 0 or args.dir_hand > 0)  # the default hands sparse waves to the tail
        kname = f"k_dirichlet_mx<{K}>" + (f" + k_dirichlet_tail<{K}>" if tail_on else "")
        rl = {"bound": "mfma" if mx else "alu", "peak": PEAK_FP16_DENSE_TFLOPS if mx else PEAK_FP32_TFLOPS,
              "unit": "TFLOP/s", "kernel": kname if mx else f"k_dirichlet<float,{K}>",
              "flop_per_particle_step": fl,
              "flop_count": "mode sum of eq. v_expand with the disk cutoff: 18 per mode + 12 per harmonic + 36",
              "peak_of": "dense FP16 matrix" if mx else "FP32 vector",
              "executed_flop_per_particle_step": flops_per_particle_step_disk(K), "velocity_engine": eng}
        traffic = other_traffic(name, eng)
        desc = ("disk-dirichlet: unit disk, 64-coefficient stream function x (1-r^2)^2, kappa=0.02, g=cos 3phi, "
                "f=-1, 25 points x 5e4 particles, dt=1e-4, walks until exit, FP32 states + FP64 exit test")
    elif name == "torus-k6-batch":
        wl = W.batch_main()
        prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
        U = torch.tensor(wl.u, dtype=torch.float64, device=dev)
        obs = torch.tensor(wl.obs, dtype=torch.float64, device=dev)
        K = int(abs(wl.modes).max())
        engine = engine_in_use(pm, args.engine, K)
        if not args.no_autotune:
            prob.autotune_time(U[0], obs, wl.kappa, wl.dt, 100_000, 1, n_probe_steps=100)

        def run():
            m, _ = prob.observe_time_batch(U, wl.n_particles, wl.seed, obs, wl.kappa, wl.T, wl.dt)
            m.cpu()
            if ctx.sync() != pm.PM_OK:
                raise pm.PMError(ctx.sync(), "forward map")
        fl = alg_flops_per_particle_step(len(wl.modes), K)
        rl = {"engine": engine}
        desc = ("torus-k6-batch: 512 pCN proposals (beta 0.2) of the |k|_inf<=6 problem in one launch, per-set "
                "particle counts log-uniform in [1e3, 1e5], 49 points, 1000 steps")
    else:
        print(f"unknown workload {name}", file=sys.stderr)
        sys.exit(2)

    elapsed, kernel_ms, work = _time_steps(run, args.steps, args.warmup, ctx)
    tail = None
    if name == "disk-dirichlet":
        steps_per_map = last["steps"]
        tail = disk_tail_bound(pm, ctx, prob, wl, u, obs, sum(kernel_ms) / len(kernel_ms) / 1e3)
    else:
        steps_per_map = work[-1]
    kern_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    if "engine" in rl:
        engine = rl["engine"]
        rl = kernel_roofline(engine, K, fl, flops_per_particle_step(K), steps_per_map, kern_s, None)
        dt_label = dtype_label(engine)
    else:
        achieved = fl * steps_per_map / kern_s / 1e12
        rl.update({"achieved": round(achieved, 3), "frac": round(achieved / rl["peak"], 4), "traffic": traffic,
                   "traffic_unit": "bytes per launch", "kernel_ms": round(kern_s * 1e3, 3),
                   "executed_tflops": round(rl["executed_flop_per_particle_step"] * steps_per_map / kern_s / 1e12,
                                            3)})
        if rl["bound"] == "mfma":
            rl["frac_of_fp32_vector_peak"] = round(achieved / PEAK_FP32_TFLOPS, 4)
        dt_label = dtype_label(rl.get("velocity_engine", "mfma"))
    out = {"metric": "particle-steps/s at 1 GPU", "value": steps_per_map * args.steps / elapsed,
           "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dt_label, "data": "synthetic",
           "config": {"workload": desc, "particle_steps_per_step": steps_per_map},
           "roofline": rl, "cpu_baseline": cpu}
    if tail is not None:
        out["tail"] = tail
    print(json.dumps(out))


def disk_tail_bound(pm, ctx, prob, wl, u, obs, map_s):
    """How far the longest walk bounds the disk map: the exit steps of one
    map (its paths), then one walker alone for as many steps as the longest
    walk took (a start at the centre with a step so small that it cannot
    leave, capped at that count), timed by the kernel's HIP events."""
    import numpy as np
    import torch
    out = prob.observe_dirichlet(u, wl.f, wl.g, obs, wl.kappa, wl.dt, wl.n_particles, wl.seed, wl.max_steps,
                                 paths=True)
    steps = out["paths"][..., 3].cpu().numpy().reshape(-1)
    ctx.sync()
    n_max = int(steps.max())
    centre = torch.zeros((1, 2), dtype=torch.float64, device=obs.device)
    prob.observe_dirichlet(u, wl.f, wl.g, centre, wl.kappa, 1e-12, 1, wl.seed, n_max)
    st = ctx.sync()
    if st not in (pm.PM_OK, pm.PM_ECAPPED):
        raise pm.PMError(st, "lone walk")
    lone_ms, lone_steps = ctx.last_kernel_stats()
    q = np.quantile(steps, [0.5, 0.95, 0.99])
    return {"exit_steps_median": float(q[0]), "exit_steps_p95": float(q[1]), "exit_steps_p99": float(q[2]),
            "exit_steps_max": n_max, "lone_walk_ms": round(lone_ms, 3), "map_ms": round(map_s * 1e3, 3),
            "lone_walk_frac_of_map": round(lone_ms / (map_s * 1e3), 4),
            "lone_walk_ns_per_step": round(lone_ms * 1e6 / max(n_max, 1), 2)}


def bench_pcn(args):
    """pCN samples/s on the main map, plain against delayed acceptance with a
    trained surrogate (a model file of `python -m paper_1808_10580_amd.da_prior
    train`), both with the particle map at 1e5 particles deciding acceptance;
    ESS of the misfit and of the first 8 coefficients (Geyer) per second,
    the equal-error comparison.  --steps is the number of chain iterations."""
    import numpy as np
    import torch
    import paper_1808_10580_amd as pm
    from paper_1808_10580_amd import da_prior, mcmc
    from paper_1808_10580_amd.surrogate import Surrogate

    if not args.model:
        print("--workload pcn needs --model (a da_prior train output)", file=sys.stderr)
        sys.exit(2)
    _, setup, wl, prior_std = da_prior._setup()
    md = np.load(args.model)
    y, gamma, beta = md["y"], float(md["gamma"]), float(md["beta"])
    ctx = pm.Context(0)
    prob, fwd = da_prior._forward(pm, ctx, wl)
    sur = Surrogate(ctx, prior_std, wl.n_obs, seed=da_prior.SEED).load(md)
    # da_aem: the stage-1 noise widened by the surrogate's held-out error
    gamma_aem = np.sqrt(gamma ** 2 + sur.err_std ** 2)
    res = {}
    for kind in ("plain", "da", "da_aem"):
        gs = gamma_aem if kind == "da_aem" else None
        c = mcmc.start_chain(setup["u_star"], fwd, y, gamma, seed=da_prior.SEED + 2,
                             surrogate=None if kind == "plain" else sur, gamma_s=gs)
        print(f"[pcn] {kind}: {args.steps} iterations", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if kind == "plain":
            mcmc.pcn_steps(c, args.steps, fwd, prior_std, y, gamma, beta)
        else:
            mcmc.da_pcn_steps(c, args.steps, fwd, sur, prior_std, y, gamma, beta, gamma_s=gs)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        S = np.array(c.samples)
        e8 = mcmc.ess_min(S, range(8))
        ephi = mcmc.ess(np.array(c.phis))
        res[kind] = {"samples_per_s": args.steps / sec, "particle_map_calls": c.n_forward,
                     "accept_rate": c.n_accept / args.steps, "ess_phi_per_s": ephi / sec,
                     "ess_min_first8_per_s": e8 / sec}
    out = {"metric": "pCN samples/s, surrogate vs plain at equal error", "value": res["da"]["samples_per_s"],
           "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": 0, "higher_is_better": True,
           "vs_baseline": None, "data": "synthetic",
           "config": {"workload": "torus-k6-fp32 posterior: y = G(u*) + N(0, 0.01^2), 1e5-particle map, pCN beta "
                                  f"{beta}, surrogate {args.model}"},
           "plain": res["plain"], "delayed_acceptance": res["da"],
           "delayed_acceptance_aem": res["da_aem"],
           "da_vs_plain": {k: {"samples_per_s": res[k]["samples_per_s"] / res["plain"]["samples_per_s"],
                               "ess_phi_per_s": res[k]["ess_phi_per_s"] / max(res["plain"]["ess_phi_per_s"], 1e-300)}
                           for k in ("da", "da_aem")}}
    print(json.dumps(out))


def mlp_train_flops(d_in: int, h: int, L: int, d_out: int, n: int) -> int:
    """Matrix-product FLOPs of one training step of the surrogate MLP (batch n,
    FMA = 2): the forward products, the weight gradients (the same shapes) and
    the input gradients of every layer but the first."""
    shapes = [(d_in, h)] + [(h, h)] * (L - 1) + [(h, d_out)]
    fwd = sum(2 * n * a * b for a, b in shapes)
    dx = sum(2 * n * a * b for a, b in shapes[1:])
    return 2 * fwd + dx


def bench_mlp(args):
    """Adam steps/s of the surrogate MLP (168 -> 512 x 3 -> 49, batch 1,024:
    the shape the delayed-acceptance study trains), and its matrix products'
    rate against the dense BF16 peak.  Timed over --steps blocks of 100
    training steps on synthetic standardised data; the rate includes the
    launch gaps between the step's kernels (their own durations: rocprofv3)."""
    import numpy as np
    import torch
    import paper_1808_10580_amd as pm

    d_in, h, L, d_out, n = 168, 512, 3, 49, 1024
    ctx = pm.Context(0)
    net = pm.MLP(ctx, d_in, h, L, d_out, n, seed=5)
    rng = np.random.default_rng(1808)
    dev = ctx.device
    X = torch.tensor(rng.standard_normal((n, d_in)), dtype=torch.float32, device=dev)
    T = torch.tensor(rng.standard_normal((n, d_out)), dtype=torch.float32, device=dev)
    per_block = 100
    for _ in range(args.warmup * per_block):
        net.train_step(X, T, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps * per_block):
        net.train_step(X, T, 1e-4)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    n_steps = args.steps * per_block
    fl = mlp_train_flops(d_in, h, L, d_out, n)
    tf = fl * n_steps / sec / 1e12
    out = {"metric": "surrogate MLP training steps/s", "value": n_steps / sec, "unit": "steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * sec / n_steps,
           "higher_is_better": True, "vs_baseline": None, "dtype": "bf16 x bf16 -> fp32", "data": "synthetic",
           "config": {"workload": f"mlp-train: {d_in} -> {h} x {L} -> {d_out}, GELU, batch {n}, Adam, "
                                  f"{per_block} steps per timed block"},
           "roofline": {"bound": "mfma", "achieved": round(tf, 3), "peak": PEAK_FP16_DENSE_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(tf / PEAK_FP16_DENSE_TFLOPS, 5), "traffic": None,
                        "flop_per_step": fl, "note": "wall time of whole training steps (launch gaps included)"}}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-particles", type=int, default=2400,
                    help="particles per point in the oracle's CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ppl", type=int, default=0, help="particles per lane (0 = library default)")
    ap.add_argument("--coef-source", type=int, default=0, help="0 = LDS, 1 = scalar cache")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the (untimed) kernel-variant autotuning before the timed steps")
    ap.add_argument("--model", default=None, help="pcn workload: a surrogate model file (da_prior train)")
    ap.add_argument("--dir-tail", type=int, default=-1,
                    help="disk walk: live lanes below which waves hand their walkers to the cooperative tail "
                         "(0 = off, -1 = library default)")
    ap.add_argument("--dir-bpc", type=int, default=0,
                    help="disk walk: persistent blocks per compute unit (0 = library default)")
    ap.add_argument("--dir-hand", type=int, default=0,
                    help="disk walk: step count at which walkers move to the cooperative tail (0 = off; "
                         "used with --dir-tail >= 0)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 512-set batched map reported beside the main line")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a known-size "
                         "kernel that calibrates the profiler's FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--engine", default="auto", choices=["auto", "valu", "mfma"],
                    help="velocity engine of FP32 problems (auto = matrix cores for torus K <= 8, disk K <= 4)")
    ap.add_argument("--workload", default="torus-k6-fp32",
                    help="torus-k6-fp32 (the benchmark line), torus-k80-turbulent, disk-dirichlet, torus-k6-batch, "
                         "torus-modes-sweep, pcn (with --model), mlp-train")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the particle map "
              "over several GPUs (one process per GPU, observations and particles split across ranks) "
              "is not built.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "torus-modes-sweep":
        bench_modes_sweep(args)
        return
    if args.workload == "mlp-train":
        bench_mlp(args)
        return
    if args.workload == "pcn":
        bench_pcn(args)
        return
    if args.workload != "torus-k6-fp32":
        bench_other(args)
        return

    import torch
    import paper_1808_10580_amd as pm
    import workloads as W

    wl = W.time_main()
    dev = torch.device("cuda", 0)
    ctx = pm.Context(0)
    ctx.set_tuning(args.ppl, args.coef_source)
    ctx.set_velocity_engine(args.engine)
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    u = torch.tensor(wl.u, dtype=torch.float64, device=dev)
    obs = torch.tensor(wl.obs, dtype=torch.float64, device=dev)
    K = int(abs(wl.modes).max())
    engine = engine_in_use(pm, args.engine, K)
    steps_per_map = wl.n_obs * wl.n_particles * wl.n_steps

    calibration_copy(torch, dev, args.copy_mib)
    tuned = None
    if not args.no_autotune and args.ppl == 0:
        # untimed setup: pick the fastest variant of the kernel this engine runs
        # (vector engine: particles per lane and coefficient source; matrix
        # cores: persistent blocks per compute unit); results are identical for all
        tuned = prob.autotune_time(u, obs, wl.kappa, wl.dt, wl.n_particles, wl.seed, n_probe_steps=100)
        ctx.set_tuning(0, 0)

    def one_map():
        m, v = prob.observe_time(u, obs, wl.kappa, wl.T, wl.dt, wl.n_particles, wl.seed)
        host = m.cpu()  # the step ends with G(u) on the host
        st = ctx.sync()
        if st != pm.PM_OK:
            raise pm.PMError(st, "forward map")
        return host

    for _ in range(args.warmup):
        one_map()
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_map()
        kernel_ms.append(ctx.last_kernel_stats()[0])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = steps_per_map * args.steps / elapsed
    print(f"[bench] {args.steps} maps in {elapsed:.3f} s; time kernel {min(kernel_ms):.2f}-"
          f"{max(kernel_ms):.2f} ms", file=sys.stderr)

    fl = alg_flops_per_particle_step(len(wl.modes), K)
    kern_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    roofline = kernel_roofline(engine, K, fl, flops_per_particle_step(K), steps_per_map, kern_s,
                               counter_traffic(engine))
    if tuned:
        roofline["variant"] = tuned
    elif engine == "valu":
        roofline["variant"] = {"particles_per_lane": args.ppl or 2, "coef_source": args.coef_source}
    batch = None if args.no_batch else measure_batch(pm, ctx, W, args)
    pcn = None if args.no_batch else measure_pcn_plain(pm, ctx, prob, wl)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, args.cpu_particles)

    out = {
        "metric": "particle-steps/s at 1 GPU",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_label(engine),
        "dtype_detail": DTYPE_DETAIL[engine],
        "data": "synthetic",
        "config": {"workload": "torus-k6-fp32: 2D torus, |k|_inf<=6 stream function (168 coefficients), "
                               "kappa=0.01, theta0 = 3 periodised Gaussian bumps, 7x7 grid x 1e5 particles, "
                               "T=1, dt=1e-3 (1000 steps), FP32 states + FP64 statistics",
                   "particle_steps_per_step": steps_per_map},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if batch is not None:
        out["batch"] = batch
    if pcn is not None:
        out["pcn_plain"] = pcn
    print(json.dumps(out))


def measure_pcn_plain(pm, ctx, prob, wl, iters: int = 40):
    """Plain pCN on this map (Section 4.1's sampler; data y = G(u*) + N(0,
    0.01^2) from a seeded prior draw u*): one captured forward map per
    iteration, u written into it, the 49 means back on the host for the
    accept test.  Samples/s over `iters` iterations after one untimed."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1808_10580_amd import mcmc
    setup = W.surrogate_setup()
    std = W.prior_std(wl.modes)
    prior_std = np.concatenate([std, std])
    fwd = mcmc.ParticleForward(prob, wl, wl.n_particles, wl.seed)
    y = fwd(setup["u_star"]) + setup["gamma"] * setup["eta"]
    c = mcmc.start_chain(setup["u_star"], fwd, y, setup["gamma"], seed=1)
    mcmc.pcn_steps(c, 1, fwd, prior_std, y, setup["gamma"], 0.04)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mcmc.pcn_steps(c, iters, fwd, prior_std, y, setup["gamma"], 0.04)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    return {"samples_per_s": iters / sec, "iterations": iters, "beta": 0.04,
            "note": "plain pCN; the surrogate comparison at equal error: bench.py --workload pcn --model ..."}


def measure_batch(pm, ctx, W, args):
    """The 512-set batch (pCN proposals of the same problem, per-set particle
    counts log-uniform in [1e3, 1e5], 5.46e11 particle-steps) in one
    persistent launch: one untimed and one timed map, beside the main line."""
    import torch
    wl = W.batch_main()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    U = torch.tensor(wl.u, dtype=torch.float64, device="cuda")
    obs = torch.tensor(wl.obs, dtype=torch.float64, device="cuda")
    K = int(abs(wl.modes).max())
    engine = engine_in_use(pm, args.engine, K)
    ms, steps = [], 0.0
    t_wall = 0.0
    for rep in range(2):
        t0 = time.perf_counter()
        m, _ = prob.observe_time_batch(U, wl.n_particles, wl.seed, obs, wl.kappa, wl.T, wl.dt)
        m.cpu()
        st = ctx.sync()
        if st != pm.PM_OK:
            raise pm.PMError(st, "batched map")
        t_wall = time.perf_counter() - t0
        k_ms, steps = ctx.last_kernel_stats()
        ms.append(k_ms)
    prob.close()
    fl = alg_flops_per_particle_step(len(wl.modes), K)
    rl = kernel_roofline(engine, K, fl, flops_per_particle_step(K), steps, ms[-1] / 1e3, None)
    return {"workload": "torus-k6-batch: 512 pCN proposals (beta 0.2), per-set particle counts log-uniform in "
                        "[1e3, 1e5], 49 points, 1000 steps, one persistent launch",
            "value": steps / t_wall, "unit": "particle-steps/s", "ms_per_map": round(1e3 * t_wall, 3),
            "particle_steps": steps, "roofline": {k: rl[k] for k in ("bound", "achieved", "peak", "frac", "kernel",
                                                                     "kernel_ms")}}


if __name__ == "__main__":
    main()
