"""The batched persistent launch and the captured forward map against the
FP64 oracle, set by set (Algorithm 1 for each parameter set u_b, with its own
particle count and seed).

  - FP64 batch of five pCN proposals with ragged particle counts
    (1, 63, 65, 129, 200): every set's means and variances equal the oracle's
    to 1e-12;
  - FP32 batch on both velocity engines: each set's means equal its single
    calls bitwise, and those calls' per-path payoffs pass the paired test
    against the oracle's paths on the same Philox streams;
  - the 512-set batch workload at its full horizon (T = 1, 1000 steps, 49
    points, per-set counts log-uniform in [1e3, 1e5]) in one launch: sets
    0, 7, 255 and 511 against an oracle subsample of 256 particles per point;
  - replays of a captured FP64 forward map, with u rewritten in place between
    them, equal the oracle's means for each u to 1e-12.
"""
import math

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


@pytest.fixture
def engine_of(ctx):
    def use(name):
        ctx.set_velocity_engine(name)
        return name
    yield use
    ctx.set_velocity_engine("auto")


def np_(t):
    return t.detach().cpu().numpy()


def tdist(a, b):
    d = np.mod(np.abs(np.asarray(a) - np.asarray(b)), 1.0)
    return np.minimum(d, 1.0 - d)


def gauss_bumps_numpy(fd, X):
    x, y = X[..., 0], X[..., 1]
    p = fd["params"]
    out = np.zeros_like(x)
    for m in range(0, len(p), 4):
        cx, cy, s, A = p[m:m + 4]
        for nx in (-1, 0, 1):
            for ny in (-1, 0, 1):
                out += A * np.exp(-((x - cx - nx) ** 2 + (y - cy - ny) ** 2) / (2 * s * s))
    return out


def test_fp64_batch_matches_oracle_per_set(pm, ctx, orc):
    wl = W.time_small()
    rng = np.random.default_rng(41)
    U = W.pcn_proposals(wl.u, wl.modes, 0.2, 5, rng)
    counts = np.array([1, 63, 65, 129, 200], dtype=np.int64)
    seeds = np.array([11, 12, 13, 2**40 + 3, 99], dtype=np.uint64)
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    mb, vb = prob.observe_time_batch(U, counts, seeds, wl.obs, wl.kappa, wl.T, wl.dt)
    assert ctx.sync() == pm.PM_OK
    mb, vb = np_(mb), np_(vb)
    worst = 0.0
    for b in range(len(counts)):
        mr, vr = orc.observe_time(wl.modes, U[b], wl.theta0, wl.obs, wl.kappa, wl.T, wl.dt, int(counts[b]),
                                  int(seeds[b]))
        worst = max(worst, np.max(np.abs(mb[b] - mr)))
        assert np.max(np.abs(mb[b] - mr)) <= 1e-12, b
        assert np.max(np.abs(vb[b] - vr)) <= 1e-12 * max(1.0, np.max(vr)), b
    print("FP64 batch of 5 sets: max |mean - oracle| %.2e" % worst)


@pytest.mark.parametrize("engine", ["valu", "mfma"])
def test_fp32_batch_paired_against_oracle(pm, ctx, orc, engine_of, engine):
    engine_of(engine)
    wl = W.time_main()
    rng = np.random.default_rng(42)
    U = W.pcn_proposals(wl.u, wl.modes, 0.2, 4, rng)
    counts = np.array([200, 333, 64, 500], dtype=np.int64)
    seeds = np.array([21, 22, 23, 24], dtype=np.uint64)
    obs = wl.obs[::7]
    T = 100 * wl.dt
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    mb, vb = prob.observe_time_batch(U, counts, seeds, obs, wl.kappa, T, wl.dt)
    assert ctx.sync() == pm.PM_OK
    mb = np_(mb)
    zs = []
    for b in range(len(counts)):
        m, v, ep = prob.observe_time(U[b], obs, wl.kappa, T, wl.dt, int(counts[b]), int(seeds[b]), endpoints=True)
        assert ctx.sync() == pm.PM_OK
        assert np.array_equal(np_(m), mb[b])
        pay, ep_ref = orc.observe_time_payoffs(wl.modes, U[b], wl.theta0, obs, wl.kappa, T, wl.dt, int(counts[b]),
                                               int(seeds[b]), endpoints=True)
        d = gauss_bumps_numpy(wl.theta0, np_(ep)) - pay
        se = d.std(axis=1, ddof=1) / math.sqrt(d.shape[1]) + 1e-300
        z = np.abs(d.mean(axis=1)) / se
        zs.append(z)
        # the kernel's means are the means of its own paths' payoffs
        assert np.allclose(mb[b], gauss_bumps_numpy(wl.theta0, np_(ep)).mean(axis=1), rtol=0, atol=1e-12)
    z = np.concatenate(zs)
    print("FP32 batch (%s), paired z over %d means: max %.2f, median endpoint error of the last set %.1e"
          % (engine, z.size, z.max(), np.median(tdist(np_(ep), ep_ref))))
    assert np.sum(z > 3) <= 1 and np.all(z < 4.5), z


def test_batch_workload_full_horizon_against_oracle_subsample(pm, ctx, orc):
    wl = W.batch_main()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    mb, vb = prob.observe_time_batch(wl.u, wl.n_particles, wl.seed, wl.obs, wl.kappa, wl.T, wl.dt)
    assert ctx.sync() == pm.PM_OK
    mb, vb = np_(mb), np_(vb)
    n_or = 256
    zs = []
    for b in (0, 7, 255, 511):
        pay = orc.observe_time_payoffs(wl.modes, wl.u[b], wl.theta0, wl.obs, wl.kappa, wl.T, wl.dt, n_or,
                                       int(wl.seed[b]))
        mr, vr = orc.mean_var(pay)
        se = np.sqrt(vr / n_or + vb[b] / wl.n_particles[b])
        zs.append(np.abs(mb[b] - mr) / se)
        # the variances: standard error of a sample variance from the fourth
        # central moment (the payoffs are far from normal: most particles
        # miss the bumps), estimated on the oracle's sample for both sides
        m4 = np.mean((pay - mr[:, None]) ** 4, axis=1)
        se_v = np.sqrt(np.maximum(m4 - vr ** 2, 0) * (1.0 / n_or + 1.0 / wl.n_particles[b]))
        assert np.all(np.abs(vb[b] - vr) <= 5 * se_v + 1e-12), (b, np.max(np.abs(vb[b] - vr) / se_v))
    z = np.concatenate(zs)
    print("512-set batch, T = 1: sets 0/7/255/511 (N_p %s) against 256 oracle particles per point: "
          "z max %.2f, %d of %d above 3" % (list(wl.n_particles[[0, 7, 255, 511]]), z.max(), np.sum(z > 3), z.size))
    assert np.sum(z > 3) <= 3 and np.all(z < 4.5), z


def test_graph_replays_match_oracle(pm, ctx, orc):
    import torch
    wl = W.time_small()
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    rng = np.random.default_rng(43)
    us = [wl.u] + [W.draw_prior(wl.modes, rng) for _ in range(2)]
    u_dev = torch.tensor(us[0], dtype=torch.float64, device="cuda")
    obs = torch.tensor(wl.obs, dtype=torch.float64, device="cuda")
    Np = 777
    g = prob.graph_time(u_dev, obs, wl.kappa, wl.T, wl.dt, Np, wl.seed)
    for r in range(2):
        for u in us:
            u_dev.copy_(torch.tensor(u, dtype=torch.float64))
            m, v = g.replay()
            assert ctx.sync() == pm.PM_OK
            mr, vr = orc.observe_time(wl.modes, u, wl.theta0, wl.obs, wl.kappa, wl.T, wl.dt, Np, wl.seed)
            assert np.max(np.abs(np_(m) - mr)) <= 1e-12
            assert np.max(np.abs(np_(v) - vr)) <= 1e-12 * np.max(vr)
    g.close()
