"""Host logic of pCN / delayed-acceptance pCN (CPU, with closed-form forward maps).

  - Phi = 0: every proposal is accepted and the chain samples the prior;
  - linear-Gaussian problem G(u) = A u: the posterior is Gaussian with
    covariance (A^T A / gamma^2 + C^-1)^-1 and mean Sigma A^T y / gamma^2;
    plain and delayed-acceptance chains both recover it, also with a widened
    (approximation-error) stage-1 noise level;
  - delayed acceptance with Phi~ = 0 reproduces plain pCN bit for bit;
  - checkpoint + resume reproduces an uninterrupted chain bit for bit;
  - the ESS estimator recovers n (1 - rho) / (1 + rho) for an AR(1) chain.
"""
import math

import numpy as np
import pytest

from paper_1808_10580_amd import mcmc


def _lin_problem(d=4, m=6, gamma=0.3, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, d))
    std = 1.0 / (1.0 + np.arange(d))
    u_star = rng.standard_normal(d) * std
    y = A @ u_star + gamma * rng.standard_normal(m)
    Cinv = np.diag(1.0 / std ** 2)
    Sigma = np.linalg.inv(A.T @ A / gamma ** 2 + Cinv)
    mu = Sigma @ A.T @ y / gamma ** 2
    return A, std, y, gamma, mu, Sigma


def test_zero_misfit_samples_the_prior():
    d = 5
    std = np.array([1.0, 0.5, 0.25, 2.0, 1.5])
    y = np.zeros(3)
    fwd = lambda u: y
    c = mcmc.start_chain(np.zeros(d), fwd, y, 1.0, seed=3)
    mcmc.pcn_steps(c, 40000, fwd, std, y, 1.0, beta=0.5)
    assert c.n_accept == 40000
    S = np.array(c.samples)[2000:]
    e = min(mcmc.ess(S[:, k]) for k in range(d))
    assert np.all(np.abs(S.mean(0)) < 5 * std / math.sqrt(e))
    assert np.all(np.abs(S.std(0) / std - 1) < 6 / math.sqrt(e))


@pytest.mark.parametrize("kind", ["plain", "da", "da_aem"])
def test_linear_gaussian_posterior(kind):
    A, std, y, gamma, mu, Sigma = _lin_problem()
    fwd = lambda u: A @ u
    # a deliberately imperfect surrogate (perturbed operator) for delayed acceptance
    A2 = A * 1.05 + 0.02
    sur = lambda u: A2 @ u
    # a widened stage-1 noise level (per observation) must not change the target
    gamma_s = gamma * np.linspace(1.0, 2.0, A.shape[0]) if kind == "da_aem" else None
    c = mcmc.start_chain(np.zeros(A.shape[1]), fwd, y, gamma, seed=11,
                         surrogate=sur if kind != "plain" else None, gamma_s=gamma_s)
    n = 60000
    if kind == "plain":
        mcmc.pcn_steps(c, n, fwd, std, y, gamma, beta=0.3)
    else:
        mcmc.da_pcn_steps(c, n, fwd, sur, std, y, gamma, beta=0.3, gamma_s=gamma_s)
        assert c.n_forward < n  # stage 1 screened some proposals
    S = np.array(c.samples)[5000:]
    sd = np.sqrt(np.diag(Sigma))
    for k in range(A.shape[1]):
        e = mcmc.ess(S[:, k])
        assert abs(S[:, k].mean() - mu[k]) < 5 * sd[k] / math.sqrt(e), (k, S[:, k].mean(), mu[k])
        assert abs(S[:, k].std() / sd[k] - 1) < 8 / math.sqrt(e)


def test_da_with_zero_surrogate_equals_plain_bitwise():
    A, std, y, gamma, mu, Sigma = _lin_problem(seed=2)
    fwd = lambda u: A @ u
    zero = lambda u: y  # Phi~ = 0
    c1 = mcmc.start_chain(np.zeros(A.shape[1]), fwd, y, gamma, seed=5)
    mcmc.pcn_steps(c1, 3000, fwd, std, y, gamma, beta=0.4)
    c2 = mcmc.start_chain(np.zeros(A.shape[1]), fwd, y, gamma, seed=5, surrogate=zero)
    mcmc.da_pcn_steps(c2, 3000, fwd, zero, std, y, gamma, beta=0.4)
    assert np.array_equal(np.array(c1.samples), np.array(c2.samples))
    assert c1.n_accept == c2.n_accept


@pytest.mark.parametrize("kind", ["plain", "da"])
def test_checkpoint_resume_is_bitwise(kind):
    A, std, y, gamma, mu, Sigma = _lin_problem(seed=4)
    fwd = lambda u: A @ u
    sur = lambda u: (A * 0.9) @ u
    run = (lambda c, n: mcmc.pcn_steps(c, n, fwd, std, y, gamma, 0.3)) if kind == "plain" else \
        (lambda c, n: mcmc.da_pcn_steps(c, n, fwd, sur, std, y, gamma, 0.3))
    c = mcmc.start_chain(np.zeros(A.shape[1]), fwd, y, gamma, seed=9, surrogate=sur)
    run(c, 2000)
    full = np.array(c.samples)
    c = mcmc.start_chain(np.zeros(A.shape[1]), fwd, y, gamma, seed=9, surrogate=sur)
    run(c, 1000)
    first = list(c.samples)
    ck = c.checkpoint()
    c2 = mcmc.Chain.resume(ck)
    run(c2, 1000)
    assert np.array_equal(np.array(first + c2.samples), full)


def test_ess_of_ar1():
    rng = np.random.default_rng(1)
    for rho in (0.0, 0.5, 0.9):
        n = 200000
        x = np.zeros(n)
        e = rng.standard_normal(n)
        for t in range(1, n):
            x[t] = rho * x[t - 1] + e[t]
        want = n * (1 - rho) / (1 + rho)
        got = mcmc.ess(x)
        assert abs(got / want - 1) < 0.12, (rho, got, want)
