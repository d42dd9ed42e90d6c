"""Batched forward maps, captured graphs and the autotuner (GPU).

  - a captured forward map replayed several times, with the program's own
    eager calls and synchronisations in between and u rewritten in place
    before each replay, equals the eager call bitwise on every replay;
  - the same for a captured batch of parameter sets;
  - the autotuner picks a valid variant and never changes results;
  - the batch of per-u particle counts and seeds equals separate calls.
Graph checks run for both FP32 velocity engines (vector FMAs and the
matrix-core contraction).
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


@pytest.fixture
def engine_of(ctx):
    def use(name):
        ctx.set_velocity_engine(name)
        return name
    yield use
    ctx.set_velocity_engine("auto")


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_graph_replays_match_eager_bitwise(pm, ctx, engine_of, engine):
    import torch
    engine_of(engine)
    wl = W.time_main()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    rng = np.random.default_rng(5)
    us = [W.draw_prior(wl.modes, rng) for _ in range(4)]
    u_dev = torch.tensor(us[0], dtype=torch.float64, device="cuda")
    obs = torch.tensor(wl.obs, dtype=torch.float64, device="cuda")
    T, Np = 0.05, 2000
    g = prob.graph_time(u_dev, obs, wl.kappa, T, wl.dt, Np, wl.seed)
    for r in range(3):
        for k, u in enumerate(us):
            u_dev.copy_(torch.tensor(u, dtype=torch.float64))
            m_g, v_g = g.replay()
            assert ctx.sync() == pm.PM_OK
            mg, vg = np_(m_g).copy(), np_(v_g).copy()
            m_e, v_e = prob.observe_time(u, wl.obs, wl.kappa, T, wl.dt, Np, wl.seed)  # eager in between
            assert ctx.sync() == pm.PM_OK
            assert np.array_equal(mg, np_(m_e)) and np.array_equal(vg, np_(v_e)), (r, k)
    assert g.particle_steps() == wl.n_obs * Np * 50
    g.close()


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_batch_graph_matches_eager(pm, ctx, engine_of, engine):
    import torch
    engine_of(engine)
    wl = W.batch_main(n_u=6, lo=100, hi=3000)
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    U = torch.tensor(wl.u, dtype=torch.float64, device="cuda").contiguous()
    obs = torch.tensor(wl.obs, dtype=torch.float64, device="cuda")
    T = 0.03
    g = prob.graph_time(U, obs, wl.kappa, T, wl.dt, wl.n_particles, wl.seed)
    for r in range(3):
        U.mul_(-1.0 if r % 2 else 1.0)
        mg, vg = g.replay()
        assert ctx.sync() == pm.PM_OK
        mg, vg = np_(mg).copy(), np_(vg).copy()
        me, ve = prob.observe_time_batch(U, wl.n_particles, wl.seed, wl.obs, wl.kappa, T, wl.dt)
        assert ctx.sync() == pm.PM_OK
        assert np.array_equal(mg, np_(me)) and np.array_equal(vg, np_(ve))


def test_autotune_picks_a_variant_and_keeps_results(pm, ctx, engine_of):
    engine_of("valu")  # the autotuner tunes the vector kernel
    wl = W.time_main()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    ctx.set_tuning(2, 0)
    m0, v0 = prob.observe_time(wl.u, wl.obs, wl.kappa, 0.05, wl.dt, 5000, wl.seed)
    m0, v0 = np_(m0).copy(), np_(v0).copy()
    ctx.set_tuning(0, 0)
    t = prob.autotune_time(wl.u, wl.obs, wl.kappa, wl.dt, 20000, n_probe_steps=20)
    print("autotune:", t)
    assert t["particles_per_lane"] in (1, 2, 3, 4) and t["coef_source"] in (0, 1) and t["probe_ms"] > 0
    m1, v1 = prob.observe_time(wl.u, wl.obs, wl.kappa, 0.05, wl.dt, 5000, wl.seed)
    assert np.array_equal(np_(m1), m0) and np.array_equal(np_(v1), v0)
    for bpc in (1, 2, 3):
        ctx.set_blocks_per_cu(bpc)
        m2, v2 = prob.observe_time(wl.u, wl.obs, wl.kappa, 0.05, wl.dt, 5000, wl.seed)
        assert np.array_equal(np_(m2), m0)
    ctx.set_blocks_per_cu(0)


def test_autotune_matrix_core_engine_keeps_results(pm, ctx, engine_of):
    """On the default matrix-core engine the autotuner picks the persistent
    grid (blocks per compute unit); the map is bitwise the same with it."""
    engine_of("auto")
    wl = W.time_main()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    m0, v0 = prob.observe_time(wl.u, wl.obs, wl.kappa, 0.05, wl.dt, 5000, wl.seed)
    m0, v0 = np_(m0).copy(), np_(v0).copy()
    t = prob.autotune_time(wl.u, wl.obs, wl.kappa, wl.dt, 20000, n_probe_steps=20)
    print("autotune (matrix cores):", t)
    assert 1 <= t["blocks_per_cu"] <= 8 and t["probe_ms"] > 0
    m1, v1 = prob.observe_time(wl.u, wl.obs, wl.kappa, 0.05, wl.dt, 5000, wl.seed)
    assert np.array_equal(np_(m1), m0) and np.array_equal(np_(v1), v0)


def test_full_batch_workload_shape(pm, ctx):
    """The 512-set batch workload (per-u particle counts log-uniform in
    [1e3, 1e5]) in one persistent launch, shortened to 20 steps: every set's
    mean equals its separate call for a sample of sets."""
    wl = W.batch_main()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    T = 20 * wl.dt
    mb, vb = prob.observe_time_batch(wl.u, wl.n_particles, wl.seed, wl.obs, wl.kappa, T, wl.dt)
    assert ctx.sync() == pm.PM_OK
    for b in (0, 7, 255, 511):
        m, v = prob.observe_time(wl.u[b], wl.obs, wl.kappa, T, wl.dt, int(wl.n_particles[b]), int(wl.seed[b]))
        assert np.array_equal(np_(m), np_(mb[b])) and np.array_equal(np_(v), np_(vb[b]))
