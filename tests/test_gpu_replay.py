"""GPU tests of pm_replay_path: one path of Algorithm 1 (eq. euler) re-run by
the forward map's own kernels, position after every step.

  R1  the last row equals the forward map's endpoint of the same (j, i) bit
      for bit, on every engine (FP64; FP32 vector units; FP32 matrix cores at
      small K; FP32 matrix cores at high K), for particles in the first,
      middle and last (ragged) chunk and for observations other than 0;
  R2  the first row is the observation point;
  R3  FP64: every row within 1e-12 of the oracle's path (orc.path);
  R4  FP32: every row within the amplification-aware FP32 path bound of the
      oracle's path, the amplification taken as the running maximum, over the
      steps so far, of the oracle's twin paths started 1e-9 away;
  plus argument validation.
"""
import numpy as np
import pytest

import workloads as W
from tests.test_gpu_time import tdist

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


@pytest.fixture
def engine_of(ctx):
    def use(name):
        ctx.set_velocity_engine(name)
        return name
    yield use
    ctx.set_velocity_engine("auto")


def np_(t):
    return t.detach().cpu().numpy()


def oracle_paths(orc, wl, modes, u, T, j, i, kicks=True):
    """The oracle's path of (j, i) and the running twin-path amplification."""
    nst = orc.n_steps(T, wl.dt)
    dte = T / nst
    x0 = np.asarray(wl.obs[j], dtype=np.float64)
    P = orc.path("torus", modes, u, wl.kappa, dte, wl.seed, i, j, x0, nst)
    A = np.zeros(nst + 1)
    if kicks:
        for kick in ((1e-9, 0.0), (0.0, 1e-9)):
            Q = orc.path("torus", modes, u, wl.kappa, dte, wl.seed, i, j, x0 + np.array(kick), nst)
            A = np.maximum(A, np.max(tdist(P, Q), axis=-1) / 1e-9)
        A = np.maximum.accumulate(A)
    return P, A


def check_replays(pm, prob, orc, wl, modes, u, T, Np, picks, fp64):
    _, _, ep = prob.observe_time(u, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed, endpoints=True)
    ep = np_(ep)
    worst = 0.0
    for j, i in picks:
        path = np_(prob.replay_path(u, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed, j, i))
        nst = pm.n_steps(T, wl.dt)
        assert path.shape == (nst + 1, 2)
        # R1: bitwise the map's endpoint
        assert np.array_equal(path[-1], ep[j, i]), (j, i, path[-1], ep[j, i])
        # R2: the start
        x0 = np.asarray(wl.obs[j], dtype=np.float64)
        assert np.max(tdist(path[0], x0)) <= (0.0 if fp64 else 2 ** -32)
        P, A = oracle_paths(orc, wl, modes, u, T, j, i, kicks=not fp64)
        err = np.max(tdist(path, P), axis=-1)
        if fp64:  # R3
            assert err.max() <= 1e-12, (j, i, err.max())
        else:     # R4
            bound = 1e-6 * np.maximum(A, 10.0)
            worst = max(worst, float(np.max(err / bound)))
            assert np.all(err <= bound), (j, i, float(np.max(err / bound)))
    print("replay: worst error / bound %.3f" % worst)


def test_fp64_replay_equals_map_and_oracle(pm, ctx, orc):
    wl = W.time_small()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    Np = 150
    picks = [(0, 0), (1, 63), (2, 64), (3, 149), (3, 128)]
    check_replays(pm, prob, orc, wl, wl.modes, wl.u, wl.T, Np, picks, fp64=True)


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_fp32_replay_small_k(pm, ctx, orc, engine_of, engine):
    engine_of(engine)
    wl = W.time_main()
    T = 40 * wl.dt
    Np = 130
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    picks = [(0, 0), (7, 65), (48, 129), (20, 127)]
    check_replays(pm, prob, orc, wl, wl.modes, wl.u, T, Np, picks, fp64=False)


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_fp32_replay_odd_step_count_full_horizon_bitwise(pm, ctx, engine_of, engine):
    """1,001 steps (odd: the last step uses the first normal pair of a
    Philox block) on the main workload: bitwise the map's endpoints."""
    engine_of(engine)
    wl = W.time_main()
    T = 1001 * wl.dt
    Np = 70
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    _, _, ep = prob.observe_time(wl.u, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed, endpoints=True)
    ep = np_(ep)
    for j, i in [(0, 69), (33, 5)]:
        path = np_(prob.replay_path(wl.u, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed, j, i))
        assert path.shape == (1002, 2)
        assert np.array_equal(path[-1], ep[j, i])


def test_fp32_replay_high_k(pm, ctx, orc):
    """|k|_inf <= 9: the high-wavenumber matrix-core kernel."""
    wl = W.time_main()
    modes = W.torus_modes(9)
    u = W.draw_prior(modes, np.random.default_rng(99))
    T = 20 * wl.dt
    Np = 100
    prob = pm.Problem(ctx, "torus", modes, theta0=wl.theta0, prec="fp32")
    picks = [(0, 3), (11, 64), (48, 99)]
    check_replays(pm, prob, orc, wl, modes, u, T, Np, picks, fp64=False)


def test_replay_rejects_bad_indices(pm, ctx):
    wl = W.time_small()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    for j, i in [(-1, 0), (wl.n_obs, 0), (0, -1), (0, 100)]:
        with pytest.raises(pm.PMError):
            prob.replay_path(wl.u, wl.obs, wl.kappa, wl.T, wl.dt, 100, wl.seed, j, i)
