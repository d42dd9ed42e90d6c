"""GPU parity of Algorithm 1 (time problem) against the FP64 oracle.

Contract (the flow is chaotic at the main workload's horizon, so full-path
agreement is checked where it is physically meaningful):
  P0  building blocks: velocity and normals against the oracle at many points;
  P1  teacher-forced single steps from oracle states: FP64 <= 1e-13,
      FP32 <= 1e-6 (torus distance);
  P2  FP64 full paths (small workload, 4 x 1000 x 100 steps): endpoints
      <= 1e-12, and the observation means equal the oracle's to 1e-12;
  P3  FP32 full paths where the oracle's twin-path amplification keeps the
      bound: <= 1e-5 at the 99th percentile on the small workload, and on
      the first 25 steps of the main workload; v = 0 paths over 1000 steps;
  P4  observation means, FP32 against the oracle on the same Philox streams:
      paired per-path differences, |mean d| <= 4 SE(d) per observation;
  plus bitwise determinism across launch shapes, batching = separate calls,
  ragged chunks, one particle, odd step counts and argument validation.
FP32 checks run for both velocity engines: the vector FMAs ("valu") and the
split-FP16 matrix-core contraction ("mfma", K <= 7), under the same bounds.
Payoffs of both sides' endpoints for P4 are evaluated in the test with numpy,
never by feeding GPU data into the oracle.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def tdist(a, b):
    d = np.abs(np.asarray(a) - np.asarray(b))
    d = np.mod(d, 1.0)
    return np.minimum(d, 1.0 - d)


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1808_10580_amd as pm
    pm.lib()
    return pm


@pytest.fixture(scope="module")
def ctx(pm):
    c = pm.Context(0)
    yield c
    c.close()


def np_(t):
    return t.detach().cpu().numpy()


@pytest.fixture
def engine_of(ctx):
    """Select a velocity engine for one test; the default is restored after."""
    def use(name):
        ctx.set_velocity_engine(name)
        return name
    yield use
    ctx.set_velocity_engine("auto")


def theta0_numpy(fd, X):
    """Test-side evaluation of the initial conditions used here."""
    x, y = X[..., 0], X[..., 1]
    p = fd["params"]
    if fd["kind"] == "sinsin":
        return p[0] * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)
    if fd["kind"] == "gauss_periodic":
        out = np.zeros_like(x)
        for m in range(0, len(p), 4):
            cx, cy, s, A = p[m:m + 4]
            for nx in (-1, 0, 1):
                for ny in (-1, 0, 1):
                    out += A * np.exp(-((x - cx - nx) ** 2 + (y - cy - ny) ** 2) / (2 * s * s))
        return out
    if fd["kind"] == "fourier":
        out = np.zeros_like(x)
        for m in range(0, len(p), 4):
            ph = 2 * np.pi * (p[m] * x + p[m + 1] * y)
            out += p[m + 2] * np.cos(ph) + p[m + 3] * np.sin(ph)
        return out
    if fd["kind"] == "gauss":
        out = np.zeros_like(x)
        for m in range(0, len(p), 4):
            out += p[m + 3] * np.exp(-p[m + 2] * ((x - p[m]) ** 2 + (y - p[m + 1]) ** 2))
        return out
    if fd["kind"] == "linear":
        return p[0] * x + p[1] * y + p[2]
    if fd["kind"] == "cos_axes":
        return p[0] * (np.cos(p[1] * x) + np.cos(p[1] * y))
    if fd["kind"] == "exp_linear":
        return np.exp(p[0] * x + p[1] * y)
    raise NotImplementedError(fd["kind"])


# ---------------------------------------------------------------------------
# P0: building blocks
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec,engine", [("fp64", "auto"), ("fp32", "valu"), ("fp32", "mfma")])
@pytest.mark.parametrize("K", [1, 2, 6, 7, 8])
def test_velocity_matches_oracle(pm, ctx, orc, engine_of, prec, engine, K):
    engine_of(engine)
    rng = np.random.default_rng(K)
    modes = W.torus_modes(K)
    u = W.draw_prior(modes, rng)
    X = rng.random((4096, 2))
    prob = pm.Problem(ctx, "torus", modes, v0=(0.25, -0.5), theta0=W.fld("zero"), prec=prec)
    V = np_(prob.velocity(u, X))
    ref = orc.velocity("torus", modes, u, X, v0=(0.25, -0.5))
    scale = np.max(np.abs(ref))
    tol = 1e-12 if prec == "fp64" else 2e-5
    print("velocity K=%d %s %s: max rel err %.2e" % (K, prec, engine, np.max(np.abs(V - ref)) / scale))
    assert np.max(np.abs(V - ref)) <= tol * scale


@pytest.mark.parametrize("prec,engine", [("fp64", "auto"), ("fp32", "valu"), ("fp32", "mfma")])
@pytest.mark.parametrize("K", [1, 4])
def test_disk_velocity_matches_oracle(pm, ctx, orc, engine_of, prec, engine, K):
    engine_of(engine)
    rng = np.random.default_rng(3 + K)
    modes = W.disk_modes() if K == 4 else W.torus_modes(K)
    u = W.draw_prior(modes, rng)
    X = W.uniform_disk_points(4096, 1.0, rng)
    prob = pm.Problem(ctx, "disk", modes, prec=prec)
    V = np_(prob.velocity(u, X))
    ref = orc.velocity("disk", modes, u, X)
    tol = 1e-12 if prec == "fp64" else 2e-5
    err = np.max(np.abs(V - ref)) / np.max(np.abs(ref))
    print("disk velocity K=%d %s %s: max rel err %.2e" % (K, prec, engine, err))
    assert err <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_normals_match_oracle(pm, ctx, orc, prec):
    rng = np.random.default_rng(1)
    n = rng.integers(0, 10**6, 50000)
    i = rng.integers(0, 2**32, 50000, dtype=np.uint64).astype(np.uint32)
    j = rng.integers(0, 49, 50000).astype(np.uint32)
    prob = pm.Problem(ctx, "torus", W.torus_modes(1), theta0=W.fld("zero"), prec=prec)
    Z = np_(prob.normals(n, i.astype(np.int64), j.astype(np.int64), seed=0xDEADBEEF12345))
    ref = orc.normals(0xDEADBEEF12345, n.astype(np.uint64), i, j)
    tol = 1e-13 if prec == "fp64" else 2e-5
    print("normals %s: max abs err %.2e" % (prec, np.max(np.abs(Z - ref))))
    assert np.max(np.abs(Z - ref)) <= tol * 6


# ---------------------------------------------------------------------------
# P1: teacher-forced steps
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("wl_name,prec,tol,engine", [("torus-k2-fp64", "fp64", 1e-13, "auto"),
                                                     ("torus-k2-fp64", "fp32", 1e-6, "valu"),
                                                     ("torus-k2-fp64", "fp32", 1e-6, "mfma"),
                                                     ("torus-k6-fp32", "fp32", 1e-6, "valu"),
                                                     ("torus-k6-fp32", "fp32", 1e-6, "mfma"),
                                                     ("torus-k6-fp32", "fp64", 1e-13, "auto")])
def test_teacher_forced_steps(pm, ctx, orc, engine_of, wl_name, prec, tol, engine):
    engine_of(engine)
    wl = W.WORKLOADS[wl_name]()
    dte = wl.T / wl.n_steps
    rows = []
    for j in range(min(wl.n_obs, 4)):
        for i in range(16):
            P = orc.path("torus", wl.modes, wl.u, wl.kappa, dte, wl.seed, i, j, wl.obs[j], wl.n_steps)
            for n in range(0, wl.n_steps, 7):
                rows.append((P[n], P[n + 1], n, i, j))
    X = np.array([r[0] for r in rows])
    Yref = np.array([r[1] for r in rows])
    n = np.array([r[2] for r in rows])
    i = np.array([r[3] for r in rows])
    j = np.array([r[4] for r in rows])
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec=prec)
    Y = np_(prob.step(wl.u, X, n, i, j, wl.kappa, dte, wl.seed))
    d = tdist(Y, Yref)
    print("teacher-forced %s %s %s: max %.2e median %.2e" % (wl_name, prec, engine, d.max(), np.median(d)))
    assert np.max(d) <= tol


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_fp32_steps_longer_than_half_the_period(pm, ctx, orc, engine_of, engine):
    """A constant drift that carries every particle 0.70 and 1.30 periods per
    step (the matrix-core engine's 32-bit fixed-point increment alone would
    overflow; its parameter set then takes the exact 64-bit-range path):
    teacher-forced steps and 20-step paths follow the oracle.  The FP32 sum
    v + v0 and the rounding of an increment of 1.3 periods carry about 1e-7
    per step."""
    engine_of(engine)
    wl = W.time_small()
    v0 = (700.3, -1301.7)
    T, Np = 20 * wl.dt, 256
    prob = pm.Problem(ctx, "torus", wl.modes, v0=v0, theta0=wl.theta0, prec="fp32")
    dte = wl.dt
    rows = []
    for j in range(wl.n_obs):
        for i in range(8):
            P = orc.path("torus", wl.modes, wl.u, wl.kappa, dte, wl.seed, i, j, wl.obs[j], 20, v0=v0)
            rows += [(P[n], P[n + 1], n, i, j) for n in range(0, 20, 3)]
    X, Yref = np.array([r[0] for r in rows]), np.array([r[1] for r in rows])
    n, i, j = (np.array([r[k] for r in rows]) for k in (2, 3, 4))
    Y = np_(prob.step(wl.u, X, n, i, j, wl.kappa, dte, wl.seed))
    d1 = tdist(Y, Yref)
    m, v, ep = prob.observe_time(wl.u, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed, endpoints=True)
    assert ctx.sync() == pm.PM_OK
    _, ep_ref = orc.observe_time_payoffs(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed,
                                         v0=v0, endpoints=True)
    err = np.max(tdist(np_(ep), ep_ref), axis=-1)
    print("steps of 0.7 / 1.3 periods, %s: teacher-forced max %.2e; 20-step paths max %.2e p99 %.2e"
          % (engine, d1.max(), err.max(), np.quantile(err, 0.99)))
    assert d1.max() <= 1e-6
    assert err.max() <= 1e-5


# ---------------------------------------------------------------------------
# P2 / P3: full paths
# ---------------------------------------------------------------------------

def test_fp64_paths_and_means_match_oracle(pm, ctx, orc):
    wl = W.time_small()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    m, v, ep = prob.observe_time(wl.u, wl.obs, wl.kappa, wl.T, wl.dt, wl.n_particles, wl.seed, endpoints=True)
    pay, ep_ref = orc.observe_time_payoffs(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, wl.T, wl.dt,
                                           wl.n_particles, wl.seed, endpoints=True)
    assert np.max(tdist(np_(ep), ep_ref)) <= 1e-12
    mr, vr = orc.mean_var(pay)
    assert np.max(np.abs(np_(m) - mr)) <= 1e-12
    assert np.max(np.abs(np_(v) - vr)) <= 1e-12 * np.max(vr)


def amplification(orc, wl, T, n_obs, n_part):
    """Oracle twin-path amplification of each path: the largest end-point
    displacement per unit start displacement for 1e-9 kicks in x and in y."""
    nst = orc.n_steps(T, wl.dt)
    dte = T / nst
    A = np.zeros((n_obs, n_part))
    for j in range(n_obs):
        for i in range(n_part):
            P = orc.path("torus", wl.modes, wl.u, wl.kappa, dte, wl.seed, i, j, wl.obs[j], nst)[-1]
            for kick in ((1e-9, 0.0), (0.0, 1e-9)):
                Q = orc.path("torus", wl.modes, wl.u, wl.kappa, dte, wl.seed, i, j, wl.obs[j] + np.array(kick),
                             nst)[-1]
                A[j, i] = max(A[j, i], np.max(tdist(P, Q)) / 1e-9)
    return A


def check_fp32_paths(err, A):
    """FP32 path contract: every path whose amplification is <= 10 ends within
    1e-5 of the oracle; beyond that the bound grows with the amplification
    (1e-6 per unit of amplification, i.e. about 1e-8 injected per step)."""
    bound = 1e-6 * np.maximum(A, 10.0)
    print("fp32 endpoint error: median %.2e p99 %.2e max %.2e; amplification median %.1f max %.1f; "
          "worst error/bound %.3f" % (np.median(err), np.quantile(err, 0.99), err.max(), np.median(A), A.max(),
                                      np.max(err / bound)))
    assert np.all(err <= bound)


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_fp32_paths_small_workload(pm, ctx, orc, engine_of, engine):
    engine_of(engine)
    wl = W.time_small()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    m, v, ep = prob.observe_time(wl.u, wl.obs, wl.kappa, wl.T, wl.dt, wl.n_particles, wl.seed, endpoints=True)
    pay, ep_ref = orc.observe_time_payoffs(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, wl.T, wl.dt,
                                           wl.n_particles, wl.seed, endpoints=True)
    err = np.max(tdist(np_(ep), ep_ref), axis=-1)
    print("all paths: p99 %.2e" % np.quantile(err, 0.99))
    assert np.quantile(err, 0.99) <= 1e-5
    A = amplification(orc, wl, wl.T, wl.n_obs, 100)
    check_fp32_paths(err[:, :100], A)
    # P4: paired mean test on the same streams
    e_gpu = theta0_numpy(wl.theta0, np_(ep))
    dd = e_gpu - pay
    se = dd.std(axis=1, ddof=1) / math.sqrt(dd.shape[1]) + 1e-300
    assert np.all(np.abs(np_(m) - pay.mean(axis=1)) <= 4 * se + 1e-12)


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_fp32_short_horizon_paths_main_workload(pm, ctx, orc, engine_of, engine):
    engine_of(engine)
    wl = W.time_main()
    T = 25 * wl.dt
    Np = 256
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    m, v, ep = prob.observe_time(wl.u, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed, endpoints=True)
    _, ep_ref = orc.observe_time_payoffs(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, T, wl.dt, Np,
                                         wl.seed, endpoints=True)
    err = np.max(tdist(np_(ep), ep_ref), axis=-1)
    assert np.quantile(err, 0.99) <= 1e-5
    A = amplification(orc, wl, T, 8, 32)
    check_fp32_paths(err[:8, :32], A)


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_fp32_zero_flow_full_horizon(pm, ctx, orc, engine_of, engine):
    engine_of(engine)
    wl = W.time_main()
    u0 = np.zeros_like(wl.u)
    Np = 200
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    _, _, ep = prob.observe_time(u0, wl.obs[:8], wl.kappa, wl.T, wl.dt, Np, wl.seed, endpoints=True)
    _, ep_ref = orc.observe_time_payoffs(wl.modes, u0, wl.theta0, wl.obs[:8], wl.kappa, wl.T, wl.dt, Np,
                                         wl.seed, endpoints=True)
    assert np.max(tdist(np_(ep), ep_ref)) <= 1e-5


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_fp32_means_main_workload_paired(pm, ctx, orc, engine_of, engine):
    """Main workload (49 points, 1000 steps), 512 particles per point: the
    per-path endpoints have decorrelated by T = 1, so this is the 3-SE test."""
    engine_of(engine)
    wl = W.time_main()
    Np = 512
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    m, v, ep = prob.observe_time(wl.u, wl.obs, wl.kappa, wl.T, wl.dt, Np, wl.seed, endpoints=True)
    pay, ep_ref = orc.observe_time_payoffs(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, wl.T, wl.dt, Np,
                                           wl.seed, endpoints=True)
    e_gpu = theta0_numpy(wl.theta0, np_(ep))
    # the GPU's own payoff and reduction reproduce the mean of its paths
    assert np.max(np.abs(np_(m) - e_gpu.mean(axis=1))) <= 1e-12
    dd = e_gpu - pay
    se = dd.std(axis=1, ddof=1) / math.sqrt(Np) + 1e-300
    z = np.abs(dd.mean(axis=1)) / se
    assert np.sum(z > 3) <= 2 and np.all(z < 4.5), z


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_full_size_means_against_oracle_subsample(pm, ctx, orc, engine_of, engine):
    """Main workload at full size (49 x 1e5 x 1000) in the benchmark's launch
    configuration; the oracle runs the first 400 particles of every point."""
    engine_of(engine)
    wl = W.time_main()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    m, v = prob.observe_time(wl.u, wl.obs, wl.kappa, wl.T, wl.dt, wl.n_particles, wl.seed)
    ctx.sync(raise_on_flags=True)
    mr, vr = orc.observe_time(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, wl.T, wl.dt, 400, wl.seed)
    se = np.sqrt(vr / 400 + np_(v) / wl.n_particles)
    z = np.abs(np_(m) - mr) / se
    assert np.sum(z > 3) <= 2 and np.all(z < 4.5), z
    # variances agree to sampling accuracy
    assert np.all(np.abs(np_(v) - vr) <= 6 * vr * math.sqrt(2 / 400) + 1e-12)


# ---------------------------------------------------------------------------
# determinism, batching, edge cases
# ---------------------------------------------------------------------------

def test_bitwise_identical_across_launch_shapes(pm, ctx, engine_of):
    wl = W.time_main()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    engine_of("valu")
    res = []
    for ppl, src in ((1, 0), (2, 0), (3, 0), (4, 0), (1, 1), (2, 1), (3, 1), (4, 1)):
        ctx.set_tuning(ppl, src)
        m, v = prob.observe_time(wl.u, wl.obs, wl.kappa, 0.2, wl.dt, 3000, wl.seed)
        res.append((np_(m), np_(v)))
    ctx.set_tuning(0, 0)
    m0, v0 = prob.observe_time(wl.u, wl.obs, wl.kappa, 0.2, wl.dt, 3000, wl.seed)
    for m, v in res:
        assert np.array_equal(m, np_(m0)) and np.array_equal(v, np_(v0))
    # the matrix-core engine: persistent grids of 1, 2, 3 blocks per CU and
    # the occupancy limit
    engine_of("mfma")
    res = []
    for bpc in (1, 2, 3, 0):
        ctx.set_blocks_per_cu(bpc)
        m, v = prob.observe_time(wl.u, wl.obs, wl.kappa, 0.2, wl.dt, 3000, wl.seed)
        res.append((np_(m), np_(v)))
    for m, v in res[:-1]:
        assert np.array_equal(m, res[-1][0]) and np.array_equal(v, res[-1][1])


def test_matrix_core_engine_falls_back_for_large_steps(pm, ctx, engine_of):
    """sqrt(2 kappa dt) above 0.05 is outside the fixed-point coordinates'
    range guarantee: the matrix-core setting then runs the vector kernel, so
    both settings give the same bits; just below the threshold they differ."""
    wl = W.time_main()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    res = {}
    for kappa in (1.5, 1.0):  # sqrt(2 kappa 1e-3) = 0.0548 and 0.0447
        for eng in ("valu", "mfma"):
            engine_of(eng)
            m, v = prob.observe_time(wl.u, wl.obs[:4], kappa, 0.02, wl.dt, 500, wl.seed)
            res[(kappa, eng)] = (np_(m), np_(v))
    assert np.array_equal(res[(1.5, "valu")][0], res[(1.5, "mfma")][0])
    assert np.array_equal(res[(1.5, "valu")][1], res[(1.5, "mfma")][1])
    assert not np.array_equal(res[(1.0, "valu")][0], res[(1.0, "mfma")][0])
    se = np.sqrt(res[(1.0, "valu")][1] / 500) + 1e-12
    assert np.all(np.abs(res[(1.0, "valu")][0] - res[(1.0, "mfma")][0]) <= 3 * se)


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_batch_equals_separate_calls_bitwise(pm, ctx, engine_of, engine):
    engine_of(engine)
    wl = W.batch_main(n_u=5, lo=50, hi=3000)
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    T = 0.1
    mb, vb = prob.observe_time_batch(wl.u, wl.n_particles, wl.seed, wl.obs, wl.kappa, T, wl.dt)
    for b in range(5):
        m, v = prob.observe_time(wl.u[b], wl.obs, wl.kappa, T, wl.dt, int(wl.n_particles[b]), int(wl.seed[b]))
        assert np.array_equal(np_(m), np_(mb[b])) and np.array_equal(np_(v), np_(vb[b]))


@pytest.mark.parametrize("Np", [1, 63, 64, 65, 129])
def test_ragged_particle_counts_fp64(pm, ctx, orc, Np):
    wl = W.time_small()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    T = 0.013  # 13 steps: odd step count
    m, v, ep = prob.observe_time(wl.u, wl.obs, wl.kappa, T, wl.dt, Np, 9, endpoints=True)
    pay, ep_ref = orc.observe_time_payoffs(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, T, wl.dt, Np, 9,
                                           endpoints=True)
    assert np.max(tdist(np_(ep), ep_ref)) <= 1e-12
    mr, vr = orc.mean_var(pay)
    assert np.allclose(np_(m), mr, rtol=0, atol=1e-12)
    if Np > 1:
        assert np.allclose(np_(v), vr, rtol=1e-10, atol=1e-14)
    else:
        assert np.all(np_(v) == 0)


@pytest.mark.parametrize("engine", ["valu", "mfma"])
@pytest.mark.parametrize("Np", [1, 63, 64, 65, 129])
def test_ragged_particle_counts_fp32(pm, ctx, orc, engine_of, engine, Np):
    """Ragged chunks and one particle on both FP32 engines: 13 steps (odd) of
    the small workload, endpoints within the FP32 path contract and the GPU's
    means equal to the mean of its own endpoints' payoffs."""
    engine_of(engine)
    wl = W.time_small()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    T = 0.013
    m, v, ep = prob.observe_time(wl.u, wl.obs, wl.kappa, T, wl.dt, Np, 9, endpoints=True)
    _, ep_ref = orc.observe_time_payoffs(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, T, wl.dt, Np, 9,
                                         endpoints=True)
    assert ep.shape[1] == Np
    assert np.max(tdist(np_(ep), ep_ref)) <= 1e-6
    e_gpu = theta0_numpy(wl.theta0, np_(ep))
    assert np.allclose(np_(m), e_gpu.mean(axis=1), rtol=0, atol=1e-12)
    if Np == 1:
        assert np.all(np_(v) == 0)


@pytest.mark.parametrize("K", [7, 8])
def test_teacher_forced_steps_largest_small_k(pm, ctx, orc, engine_of, K):
    """The largest cutoffs of the small-K matrix-core path in teacher-forced
    steps against the oracle: K = 7 (B = 15 of 16 tile entries) and K = 8
    (the tile plus the entry-16 row and column on the vector units)."""
    engine_of("mfma")
    modes = W.torus_modes(K)
    rng = np.random.default_rng(70 + K)
    u = W.draw_prior(modes, rng)
    kappa, dt, seed = 0.01, 1e-3, 5
    X = rng.random((700, 2))
    n = rng.integers(0, 1000, 700)
    i = rng.integers(0, 10**5, 700)
    j = rng.integers(0, 49, 700)
    prob = pm.Problem(ctx, "torus", modes, theta0=W.fld("zero"), prec="fp32")
    Y = np_(prob.step(u, X, n, i, j, kappa, dt, seed))
    Yr = orc.step("torus", modes, u, kappa, dt, seed, X, n, i, j)
    d = tdist(Y, Yr)
    print("teacher-forced K=%d mfma: max %.2e" % (K, d.max()))
    assert np.max(d) <= 1e-6


def test_empty_mode_table_is_pure_diffusion(pm, ctx, orc):
    prob = pm.Problem(ctx, "torus", np.zeros((0, 2), np.int32), theta0=W.fld("sinsin", [1.0]), prec="fp64")
    obs = np.array([[0.1, 0.3], [0.7, 0.2]])
    m, v, ep = prob.observe_time(np.zeros(0), obs, 0.05, 0.1, 1e-3, 300, 4, endpoints=True)
    pay, ep_ref = orc.observe_time_payoffs(np.zeros((0, 2), np.int32), np.zeros(0), W.fld("sinsin", [1.0]), obs,
                                           0.05, 0.1, 1e-3, 300, 4, endpoints=True)
    assert np.max(tdist(np_(ep), ep_ref)) <= 1e-12


THETA0_KINDS = {
    "fourier": W.fld("fourier", [1, 0, 0.3, -0.2, 1, 2, 0.1, 0.4]),
    "gauss": W.fld("gauss", [0.4, 0.6, 8.0, 1.5]),
    "linear": W.fld("linear", [0.5, -0.25, 0.1]),
    "cos_axes": W.fld("cos_axes", [0.5, 2.0]),
    "exp_linear": W.fld("exp_linear", [0.3, -0.7]),
}


@pytest.mark.parametrize("kind", list(THETA0_KINDS))
@pytest.mark.parametrize("prec,engine", [("fp64", "auto"), ("fp32", "valu"), ("fp32", "mfma")])
def test_theta0_kinds_against_oracle(pm, ctx, orc, engine_of, kind, prec, engine):
    """Initial conditions of other kinds: the means are those of theta0 (a
    test-side formula) at the GPU's own endpoints, the endpoints follow the
    oracle's paths, and in FP64 the means equal the oracle's to 1e-12."""
    engine_of(engine)
    wl = W.time_small()
    th = THETA0_KINDS[kind]
    Np = 130
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=th, prec=prec)
    m, v, ep = prob.observe_time(wl.u, wl.obs, wl.kappa, wl.T, wl.dt, Np, wl.seed, endpoints=True)
    pay, ep_ref = orc.observe_time_payoffs(wl.modes, wl.u, th, wl.obs, wl.kappa, wl.T, wl.dt, Np, wl.seed,
                                           endpoints=True)
    mr, vr = orc.mean_var(pay)
    # the payoff route: the means are those of theta0 at the GPU's own endpoints
    e_gpu = theta0_numpy(th, np_(ep))
    assert np.max(np.abs(np_(m) - e_gpu.mean(axis=1))) <= 1e-12 * (1.0 + np.max(np.abs(e_gpu)))
    assert np.max(np.abs(np_(v) - e_gpu.var(axis=1, ddof=1))) <= 1e-12 * (1.0 + np.max(e_gpu ** 2))
    if prec == "fp64":
        assert np.max(tdist(np_(ep), ep_ref)) <= 1e-12
        assert np.max(np.abs(np_(m) - mr)) <= 1e-12
        assert np.max(np.abs(np_(v) - vr)) <= 1e-12 * max(np.max(vr), 1e-300) + 1e-300
    else:
        assert np.quantile(np.max(tdist(np_(ep), ep_ref), axis=-1), 0.99) <= 1e-5
    assert ctx.sync() == pm.PM_OK


def test_invalid_arguments_raise(pm, ctx):
    wl = W.time_small()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    for bad in (dict(kappa=-1.0), dict(T=0.0), dict(dt=0.0), dict(n_particles=0)):
        kw = dict(kappa=wl.kappa, T=wl.T, dt=wl.dt, n_particles=10)
        kw.update(bad)
        with pytest.raises(pm.PMError) as e:
            prob.observe_time(wl.u, wl.obs, kw["kappa"], kw["T"], kw["dt"], kw["n_particles"], 1)
        assert e.value.status == pm.PM_EINVAL
    with pytest.raises(pm.PMError):  # beyond every compiled path
        pm.Problem(ctx, "torus", np.array([[96, 0]], np.int32), theta0=wl.theta0)
    with pytest.raises(pm.PMError):  # FP64 has only the vector path (|k| <= 8)
        pm.Problem(ctx, "torus", np.array([[9, 0]], np.int32), theta0=wl.theta0, prec="fp64")
    dprob = pm.Problem(ctx, "disk", W.disk_modes())
    with pytest.raises(pm.PMError):
        dprob.observe_time(np.zeros(64), wl.obs, 0.1, 1.0, 0.1, 10, 1)
    assert ctx.sync() == pm.PM_OK
