"""GPU parity of the high-wavenumber path (|k| > 8: velocity on the matrix
cores in split FP16) against the FP64 oracle, which sums eq. v_expand mode by
mode with its own sin/cos.

  P0  velocity at scattered points (ragged wave counts) for square and
      Euclidean-ball mode sets up to |k| = 95, within the FP32 contract
      2e-5 |v|max (split FP16 is expected near 5e-7);
  P1  teacher-forced Euler-Maruyama steps of the turbulent workload
      (|k|_2 <= 80) within 1e-6 on the torus;
  P3  FP32 paths over the first 20 steps within the amplification-aware bound;
  P4  multi-time means at 128 particles per point against the oracle's per-time
      runs on the same Philox streams, and the full workload (2 x 1e5 x 4,800
      steps, 13 readouts) against an oracle subsample;
  plus bitwise: a batch equals separate calls and a graph replay equals the
  eager call.
"""
import numpy as np
import pytest

import workloads as W
from tests.test_gpu_time import amplification, check_fp32_paths, tdist

pytestmark = pytest.mark.gpu


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


MODE_SETS = {
    "square9": lambda: W.torus_modes(9),
    "square16": lambda: W.torus_modes(16),
    "ball40": lambda: W.half_plane(W.l2_ball_modes(40.0)),
    "ball80": lambda: W.half_plane(W.l2_ball_modes(80.0)),
    "square95": lambda: W.torus_modes(95),
}


@pytest.mark.parametrize("name", list(MODE_SETS))
def test_velocity_matches_oracle(pm, ctx, orc, name):
    modes = MODE_SETS[name]()
    rng = np.random.default_rng(list(MODE_SETS).index(name) + 40)
    u = W.draw_prior(modes, rng)
    X = rng.random((1000, 2))
    X[:3] = [[0.0, 0.0], [0.5, 0.5], [0.999999, 1e-7]]
    prob = pm.Problem(ctx, "torus", modes, prec="fp32")
    V = np_(prob.velocity(u, X))
    Vr = orc.velocity("torus", modes, u, X)
    err = np.max(np.abs(V - Vr)) / np.max(np.abs(Vr))
    print("%s (%d modes): velocity error / |v|max = %.2e" % (name, len(modes), err))
    assert err <= 2e-5
    prob.close()


def test_drift_and_zero_field(pm, ctx, orc):
    modes = W.torus_modes(12)
    X = np.random.default_rng(3).random((70, 2))
    prob = pm.Problem(ctx, "torus", modes, v0=(0.3, -0.7), prec="fp32")
    V = np_(prob.velocity(np.zeros(2 * len(modes)), X))
    assert np.array_equal(V, np.broadcast_to(np.array([0.3, -0.7], dtype=np.float32).astype(np.float64), V.shape))
    prob.close()


def test_teacher_forced_steps(pm, ctx, orc):
    wl = W.turbulent_k80()
    rng = np.random.default_rng(5)
    cnt = 777
    X = rng.random((cnt, 2))
    n = rng.integers(0, 4800, cnt)
    i = rng.integers(0, 100_000, cnt)
    j = rng.integers(0, 2, cnt)
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    Y = np_(prob.step(wl.u, X, n, i, j, wl.kappa, wl.dt, wl.seed))
    Yr = orc.step("torus", wl.modes, wl.u, wl.kappa, wl.dt, wl.seed, X, n, i, j)
    err = np.max(tdist(Y, Yr))
    print("teacher-forced step error %.2e" % err)
    assert err <= 1e-6
    prob.close()


def test_fp32_short_paths(pm, ctx, orc):
    wl = W.turbulent_k80()
    T = 20 * wl.dt
    Np = 64
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    _, _, ep = prob.observe_time(wl.u, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed, endpoints=True)
    _, ep_ref = orc.observe_time_payoffs(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed,
                                         endpoints=True)
    err = np.max(tdist(np_(ep), ep_ref), axis=-1)
    A = amplification(orc, wl, T, 2, 16)
    check_fp32_paths(err[:, :16], A)
    assert np.quantile(err, 0.99) <= 1e-5
    prob.close()


def test_multitime_means_against_oracle(pm, ctx, orc):
    wl = W.turbulent_k80()
    steps = [0, 100, 200, 400]
    Np = 128
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    m, v = prob.observe_time_multi(wl.u, wl.obs, wl.kappa, steps, wl.dt, Np, wl.seed)
    mr, vr = orc.observe_time_multi(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, steps, wl.dt, Np, wl.seed)
    # read 0 is theta0 at the points: no randomness
    assert np.allclose(np_(m)[0], mr[0], rtol=0, atol=1e-6)
    # Both sides follow the same Philox streams, so the difference of the means
    # is sampling noise of the path errors plus the path errors themselves; the
    # allowance 1e-5 covers FP32 path errors of ~1.7e-6 times theta0's largest
    # slope (about 6 for unit bumps of width 0.1).
    se = np.sqrt((np_(v) + vr) / Np)
    d = np.abs(np_(m) - mr)[1:]
    print("k80 multi-time: max |d| %.2e, max z %.2f" % (d.max(), (d / (se[1:] + 1e-300)).max()))
    assert np.all(d <= 4.5 * se[1:] + 1e-5), (d, se)
    prob.close()


def test_full_turbulent_workload_against_oracle_subsample(pm, ctx, orc):
    """The turbulent workload at full size (2 points x 1e5 particles x 4,800
    steps, 13 readouts) against 24 oracle particles per point."""
    wl = W.turbulent_k80()
    reads = wl.extra["read_steps"]
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    m, v = prob.observe_time_multi(wl.u, wl.obs, wl.kappa, reads, wl.dt, wl.n_particles, wl.seed)
    ctx.sync(raise_on_flags=True)
    n_or = 24
    mr, vr = orc.observe_time_multi(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, reads[:4], wl.dt, n_or, wl.seed)
    assert np.allclose(np_(m)[0], mr[0], rtol=0, atol=1e-12)  # read 0: theta0 at the points
    se = np.sqrt(vr / n_or + np_(v)[:4] / wl.n_particles)[1:]
    z = np.abs(np_(m)[1:4] - mr[1:]) / (se + 1e-300)
    print("full k80 vs oracle subsample: max z %.2f" % z.max())
    assert np.all(z < 4.5), z
    assert np.all(np.isfinite(np_(m))) and np.all(np_(v) >= 0)
    prob.close()


def test_batch_equals_separate_calls_bitwise(pm, ctx):
    wl = W.turbulent_k80()
    rng = np.random.default_rng(9)
    U = np.stack([wl.u, W.draw_prior(wl.modes, rng), W.draw_prior(wl.modes, rng)])
    nps = [100, 64, 129]
    seeds = [7, 8, 9]
    T = 30 * wl.dt
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    mb, vb = prob.observe_time_batch(U, nps, seeds, wl.obs, wl.kappa, T, wl.dt)
    for b in range(3):
        m, v = prob.observe_time(U[b], wl.obs, wl.kappa, T, wl.dt, nps[b], seeds[b])
        assert np.array_equal(np_(m), np_(mb[b])) and np.array_equal(np_(v), np_(vb[b]))
    prob.close()


def test_graph_replay_equals_eager(pm, ctx):
    import torch
    wl = W.turbulent_k80()
    T = 30 * wl.dt
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    u = torch.tensor(wl.u, dtype=torch.float64, device="cuda")
    obs = torch.tensor(wl.obs, dtype=torch.float64, device="cuda")
    m0, v0 = prob.observe_time(u, obs, wl.kappa, T, wl.dt, 500, wl.seed)
    m0, v0 = np_(m0), np_(v0)
    g = prob.graph_time(u, obs, wl.kappa, T, wl.dt, 500, wl.seed)
    for _ in range(3):
        m_g, v_g = g.replay()
        ctx.sync(raise_on_flags=True)
        assert np.array_equal(np_(m_g).reshape(-1), m0) and np.array_equal(np_(v_g).reshape(-1), v0)
        prob.observe_time(u, obs, wl.kappa, T / 2, wl.dt, 100, 3)  # eager work between replays
        ctx.sync()
    g.close()
    prob.close()


def test_high_k_limits(pm, ctx):
    with pytest.raises(pm.PMError):  # beyond the matrix-core path
        pm.Problem(ctx, "torus", np.array([[96, 0]]), prec="fp32")
    with pytest.raises(pm.PMError):  # FP64 keeps the vector path's limit
        pm.Problem(ctx, "torus", np.array([[9, 0]]), prec="fp64")
    with pytest.raises(pm.PMError):  # a wavevector listed twice
        pm.Problem(ctx, "torus", np.array([[9, 0], [9, 0]]), prec="fp32")
