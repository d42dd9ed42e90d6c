"""GPU parity of the multi-time readout (one ensemble per point read out as
it passes t_k = n_k dt) against the oracle's definition (Algorithm 1 run once
per (t_k, x_j) with step dt and the same seed).

  - FP64, small workload: every mean and variance within 1e-12 of the
    oracle's, read steps including 0, odd and even counts;
  - each readout equals a single-time call to T = n_k dt bit for bit (dt a
    power of two, so T / N_t gives back dt exactly), FP64 and FP32;
  - FP32, main workload, 512 particles: |G_gpu - G_oracle| within the
    standard errors at every time (paths decorrelate by T = 1);
  - ragged particle counts and argument validation.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

DT = 2.0 ** -10


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


@pytest.mark.parametrize("steps,Np", [([0, 7, 40, 101], 1000), ([1, 2, 3], 65), ([64], 129)])
def test_fp64_matches_oracle(pm, ctx, orc, steps, Np):
    wl = W.time_small()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    m, v = prob.observe_time_multi(wl.u, wl.obs, wl.kappa, steps, DT, Np, wl.seed)
    mr, vr = orc.observe_time_multi(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, steps, DT, Np, wl.seed)
    assert m.shape == (len(steps), wl.n_obs)
    assert np.max(np.abs(np_(m) - mr)) <= 1e-12
    assert np.max(np.abs(np_(v) - vr)) <= 1e-12 * max(np.max(vr), 1e-300) + 1e-300
    prob.close()


@pytest.mark.parametrize("prec,engine", [("fp64", "auto"), ("fp32", "valu"), ("fp32", "mfma")])
def test_each_readout_equals_a_single_time_call(pm, ctx, prec, engine):
    ctx.set_velocity_engine(engine)
    wl = W.time_main()
    steps = [0, 1, 50, 123, 300]
    Np = 700
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec=prec)
    m, v = prob.observe_time_multi(wl.u, wl.obs, wl.kappa, steps, DT, Np, wl.seed)
    for k, n in enumerate(steps):
        if n == 0:
            continue  # a single-time call needs T > 0
        m1, v1 = prob.observe_time(wl.u, wl.obs, wl.kappa, n * DT, DT, Np, wl.seed)
        assert np.array_equal(np_(m[k]), np_(m1)) and np.array_equal(np_(v[k]), np_(v1)), (prec, n)
    prob.close()
    ctx.set_velocity_engine("auto")


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_fp32_means_main_workload(pm, ctx, orc, engine):
    ctx.set_velocity_engine(engine)
    wl = W.time_main()
    steps = [250, 500, 1000]
    Np = 512
    dt = wl.dt
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    m, v = prob.observe_time_multi(wl.u, wl.obs, wl.kappa, steps, dt, Np, wl.seed)
    mr, vr = orc.observe_time_multi(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, steps, dt, Np, wl.seed)
    se = np.sqrt((np_(v) + vr) / Np) + 1e-300
    z = np.abs(np_(m) - mr) / se
    print("multi-time fp32 %s: max z %.2f" % (engine, z.max()))
    ctx.set_velocity_engine("auto")
    assert np.sum(z > 3) <= 3 and np.all(z < 4.5), z
    prob.close()


def test_invalid_read_lists_raise(pm, ctx):
    wl = W.time_small()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    for bad in ([], [5, 5], [5, 3], [-1, 2], list(range(1, 66))):
        with pytest.raises(pm.PMError):
            prob.observe_time_multi(wl.u, wl.obs, wl.kappa, bad, DT, 10, wl.seed)
    with pytest.raises(pm.PMError):
        prob.observe_time_multi(wl.u, wl.obs, wl.kappa, [1, 2], 0.0, 10, wl.seed)
    prob.close()
