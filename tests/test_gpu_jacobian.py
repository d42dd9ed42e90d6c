"""GPU finite-difference Jacobian of G (one batched launch of the 4M
perturbed maps, common random numbers) against the oracle's definition.

  - FP64 small workload: every entry within 1e-7 of the oracle's Jacobian
    (the FP64 maps agree to ~1e-12, divided by the step 2h = 2e-4);
  - FP32 main workload: each column equals the difference of two separate
    single-map calls bit for bit (the batch reproduces separate calls);
  - a high-wavenumber problem (|k| = 9) through the same entry point;
  - a non-positive step is rejected.
"""
import numpy as np
import pytest

import workloads as W

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


def test_fp64_jacobian_matches_oracle(pm, ctx, orc):
    wl = W.time_small()
    obs = wl.obs[:3]
    T, Np, h = 0.02, 200, 1e-4
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    J = np_(prob.jacobian_time(wl.u, obs, wl.kappa, T, wl.dt, Np, wl.seed, h))
    Jr = orc.jacobian_time(wl.modes, wl.u, wl.theta0, obs, wl.kappa, T, wl.dt, Np, wl.seed, h)
    assert J.shape == Jr.shape == (3, 2 * len(wl.modes))
    print("fp64 Jacobian: max |J - J_oracle| %.2e, max |J| %.2e" % (np.max(np.abs(J - Jr)), np.max(np.abs(Jr))))
    assert np.max(np.abs(J - Jr)) <= 1e-7
    assert np.max(np.abs(Jr)) > 1e-2
    prob.close()


@pytest.mark.parametrize("modes_name,engine", [("k6", "valu"), ("k6", "mfma"), ("k9", "auto")])
def test_columns_equal_separate_calls_bitwise(pm, ctx, modes_name, engine):
    ctx.set_velocity_engine(engine)
    wl = W.time_main()
    modes = wl.modes if modes_name == "k6" else W.torus_modes(9)
    u = wl.u if modes_name == "k6" else W.draw_prior(modes, np.random.default_rng(2))
    T, Np, h = 20 * wl.dt, 300, 1e-3
    prob = pm.Problem(ctx, "torus", modes, theta0=wl.theta0, prec="fp32")
    J = np_(prob.jacobian_time(u, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed, h))
    for k in (0, 7, u.size - 1):
        up, um = u.copy(), u.copy()
        up[k] = u[k] + h
        um[k] = u[k] - h
        mp, _ = prob.observe_time(up, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed)
        mm, _ = prob.observe_time(um, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed)
        col = (np_(mp) - np_(mm)) / (up[k] - um[k])
        assert np.array_equal(J[:, k], col), (modes_name, k)
    prob.close()
    ctx.set_velocity_engine("auto")


def test_invalid_step_raises(pm, ctx):
    wl = W.time_small()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    for h in (0.0, -1e-3, float("nan")):
        with pytest.raises(pm.PMError):
            prob.jacobian_time(wl.u, wl.obs, wl.kappa, wl.T, wl.dt, 10, 1, h)
    prob.close()
