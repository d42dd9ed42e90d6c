"""pCN over the HIP particle map (Section 4.1: the paper samples its
posteriors with pCN, one forward map per proposal).

  - a plain pCN chain whose forward map is the HIP map (a captured FP64 graph
    replay, 4 points x 256 particles x 100 steps, common random numbers) and
    the same chain whose forward map is the FP64 oracle take the same
    accept/reject decisions at every iteration, with misfits equal to 1e-9
    relative;
  - delayed acceptance with a zero stage-1 misfit over the HIP map reproduces
    plain pCN over the HIP map bit for bit.
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


def _setup(pm, orc):
    from paper_1808_10580_amd import mcmc
    wl = W.time_small()
    Np, seed, gamma = 256, 5, 0.05
    rng = np.random.default_rng(77)
    u_star = W.draw_prior(wl.modes, rng)
    y = orc.observe_time(wl.modes, u_star, wl.theta0, wl.obs, wl.kappa, wl.T, wl.dt, 4096, 9)[0]
    y = y + gamma * rng.standard_normal(y.shape)
    std = np.concatenate([W.prior_std(wl.modes)] * 2)  # per coefficient: a then b
    ctx = pm.Context(0)
    prob = pm.Problem(ctx, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    hip = mcmc.ParticleForward(prob, wl, Np, seed)

    def oracle_map(u):
        return orc.observe_time(wl.modes, u, wl.theta0, wl.obs, wl.kappa, wl.T, wl.dt, Np, seed)[0]
    return mcmc, wl, ctx, prob, hip, oracle_map, y, std, gamma


def test_plain_pcn_on_the_hip_map_follows_the_oracle_map(pm, orc):
    mcmc, wl, ctx, prob, hip, oracle_map, y, std, gamma = _setup(pm, orc)
    n, beta = 40, 0.3
    a = mcmc.start_chain(np.zeros(len(std)), hip, y, gamma, seed=123)
    mcmc.pcn_steps(a, n, hip, std, y, gamma, beta)
    b = mcmc.start_chain(np.zeros(len(std)), oracle_map, y, gamma, seed=123)
    mcmc.pcn_steps(b, n, oracle_map, std, y, gamma, beta)
    pa, pb = np.array(a.phis), np.array(b.phis)
    acc_a = [not np.array_equal(a.samples[k], a.samples[k - 1]) for k in range(1, n)]
    acc_b = [not np.array_equal(b.samples[k], b.samples[k - 1]) for k in range(1, n)]
    rel = np.max(np.abs(pa - pb) / np.maximum(1.0, np.abs(pb)))
    print("pCN x%d on the HIP map vs the oracle map: %d accepts each; max relative misfit difference %.2e"
          % (n, a.n_accept, rel))
    assert a.n_accept == b.n_accept and acc_a == acc_b
    assert a.n_accept > 0
    assert rel <= 1e-9
    assert np.max(np.abs(np.array(a.samples) - np.array(b.samples))) == 0.0
    prob.close()
    ctx.close()


def test_delayed_acceptance_with_zero_surrogate_misfit_is_plain_pcn_on_the_hip_map(pm, orc):
    mcmc, wl, ctx, prob, hip, oracle_map, y, std, gamma = _setup(pm, orc)
    n, beta = 60, 0.3
    a = mcmc.start_chain(np.zeros(len(std)), hip, y, gamma, seed=321)
    mcmc.pcn_steps(a, n, hip, std, y, gamma, beta)
    zero = lambda u: y  # stage-1 misfit 0 for every proposal
    b = mcmc.start_chain(np.zeros(len(std)), hip, y, gamma, seed=321, surrogate=zero)
    mcmc.da_pcn_steps(b, n, hip, zero, std, y, gamma, beta)
    assert a.n_accept == b.n_accept and b.n_forward == n
    assert np.array_equal(np.array(a.samples), np.array(b.samples))
    assert a.phis == b.phis
    prob.close()
    ctx.close()
