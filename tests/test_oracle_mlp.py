"""Pins of the FP64 MLP oracle (surrogate of the forward map).

GELU is checked against x * Phi(x) from scipy's normal CDF and its derivative
against finite differences; the full backward pass against central finite
differences of the loss on a small network (relative 1e-7).
"""
import numpy as np
from scipy.stats import norm

from oracle import mlp


def test_gelu_is_x_times_normal_cdf():
    z = np.linspace(-6, 6, 1001)
    assert np.allclose(mlp.gelu(z), z * norm.cdf(z), rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, rtol=1e-8, atol=1e-9)


def test_backward_matches_finite_differences():
    dims = (6, 9, 3, 4)
    rng = np.random.default_rng(0)
    p = mlp.init_params(dims, 1) + 0.1 * rng.standard_normal(mlp.n_params(*dims))
    x = rng.standard_normal((5, 6))
    t = rng.standard_normal((5, 4))
    scale = rng.uniform(0.5, 2, 6)
    mu, sd = rng.standard_normal(4), rng.uniform(0.5, 2, 4)
    loss, g = mlp.loss_and_grads(p, dims, x, t, scale, mu, sd)
    fd = np.zeros_like(p)
    h = 1e-6
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = h
        lp, _ = mlp.loss_and_grads(p + e, dims, x, t, scale, mu, sd)
        lm, _ = mlp.loss_and_grads(p - e, dims, x, t, scale, mu, sd)
        fd[k] = (lp - lm) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-7 * np.linalg.norm(fd)


def test_parameter_count_of_the_surrogate():
    # 168 -> 512 -> 512 -> 512 -> 49
    assert mlp.n_params(168, 512, 3, 49) == 636977
