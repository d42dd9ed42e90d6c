"""Pins of the FP64 MLP oracle (surrogate of the forward map).

GELU is checked against x * Phi(x) from scipy's normal CDF and its derivative
against finite differences; the full backward pass against central finite
differences of the loss on a small network (relative 1e-7).

Adam (Kingma and Ba 2015) is pinned by what its definition fixes without
re-deriving its update:
  A1  a constant gradient g gives bias-corrected moments equal to g and g^2 at
      every step, so each step moves a weight by exactly lr g / (|g| + eps)
      (a missing or wrong bias correction moves it by another amount);
  A2  zero gradients never move a weight; the moments of other weights do not
      leak into it (each coordinate is its own optimiser);
  A3  eps enters outside the square root: a gradient of 1e-10 moves a weight
      by lr / 101 on the first step (eps inside the root would give 0.0099);
  A4  rescaling the loss by c > 0 leaves the steps unchanged (eps aside);
  A5  a single gradient spike after t - 1 zero gradients moves the weight by
      lr (1 - beta1) sqrt(1 - beta2^t) / ((1 - beta1^t) sqrt(1 - beta2)),
      (lr itself at t = 1), never more than the bound lr (1 - beta1) /
      sqrt(1 - beta2) of the paper's Section 2.1, which it approaches as t
      grows;
  A6  on a quadratic the first step is lr sign(g) and Adam drives the weight
      to the minimum.
"""
import numpy as np
import pytest
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


def _run_adam(grad_fn, p0, steps, lr):
    p, m1, m2 = np.array(p0, dtype=np.float64), np.zeros(len(p0)), np.zeros(len(p0))
    path = [p.copy()]
    for t in range(1, steps + 1):
        p, m1, m2 = mlp.adam_update(p, grad_fn(p, t), m1, m2, t, lr)
        path.append(p.copy())
    return np.array(path)


def test_A1_constant_gradient_steps_are_exact():
    g = np.array([0.3, -2.0, 5e-3, 7.0])
    lr = 1e-3
    path = _run_adam(lambda p, t: g, np.zeros(4), 50, lr)
    step = lr * g / (np.abs(g) + 1e-8)
    for t in range(1, 51):
        assert np.allclose(path[t] - path[t - 1], -step, rtol=1e-12, atol=0)


def test_A2_zero_gradient_and_independent_coordinates():
    rng = np.random.default_rng(3)
    G = rng.standard_normal((20, 3))
    G[:, 1] = 0.0
    full = _run_adam(lambda p, t: G[t - 1], np.ones(3), 20, 1e-2)
    assert np.all(full[:, 1] == 1.0)
    # coordinate 0 alone follows the same path as inside the vector
    alone = _run_adam(lambda p, t: G[t - 1, :1], np.ones(1), 20, 1e-2)
    assert np.array_equal(alone[:, 0], full[:, 0])


def test_A3_eps_outside_the_square_root():
    p, _, _ = mlp.adam_update(np.zeros(1), np.array([1e-10]), np.zeros(1), np.zeros(1), 1, 1.0)
    assert abs(-p[0] - 1.0 / 101.0) < 1e-12


def test_A4_loss_scale_invariance():
    rng = np.random.default_rng(4)
    G = rng.standard_normal((30, 5))
    a = _run_adam(lambda p, t: G[t - 1], np.zeros(5), 30, 1e-3)
    b = _run_adam(lambda p, t: 1e3 * G[t - 1], np.zeros(5), 30, 1e-3)
    assert np.allclose(a, b, rtol=0, atol=1e-9)


def test_A5_sparse_spike_approaches_the_step_bound():
    lr, b1, b2 = 1.0, 0.9, 0.999
    bound = lr * (1 - b1) / np.sqrt(1 - b2)
    step = 0.0
    for t in (1, 10, 100, 1000, 10000):
        seq = np.zeros(t)
        seq[-1] = 2.5e4  # eps negligible
        path = _run_adam(lambda p, s: np.array([seq[s - 1]]), np.zeros(1), t, lr)
        step = -(path[-1, 0] - path[-2, 0])
        expect = lr * (1 - b1) * np.sqrt(1 - b2 ** t) / ((1 - b1 ** t) * np.sqrt(1 - b2))
        assert abs(step - expect) < 1e-9 * expect
        assert step <= bound * (1 + 1e-12)
        if t == 1:
            assert abs(step - lr) < 1e-9
    assert step > 0.99 * bound


def test_A6_quadratic():
    h = np.array([2.0, 0.5, 10.0])
    p0 = np.array([1.0, -3.0, 0.2])
    path = _run_adam(lambda p, t: h * p, p0, 4000, 1e-2)
    assert np.allclose(path[1] - p0, -1e-2 * np.sign(h * p0), rtol=1e-6)
    assert np.all(np.abs(path[-1]) < 2e-2)


# ---------------------------------------------------------------------------
# The element-wise BF16 tolerances that the GPU tests apply (tests/mlp_bounds.py)
# ---------------------------------------------------------------------------

def _bounds_case(dims, n, seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(dims, seed) + 0.02 * rng.standard_normal(mlp.n_params(*dims))
    x = rng.standard_normal((n, dims[0]))
    t = rng.standard_normal((n, dims[3]))
    scale = rng.uniform(0.5, 2.0, dims[0])
    mu, sd = rng.standard_normal(dims[3]), rng.uniform(0.5, 2.0, dims[3])
    return p, x, t, scale, mu, sd


@pytest.mark.parametrize("dims,n", [((8, 16, 2, 4), 50), ((168, 512, 3, 49), 64)])
def test_bf16_tolerances_cover_an_emulation_of_the_rounding(dims, n):
    """The GPU's rounding sequence emulated in numpy stays within 3/4 of the
    element-wise tolerances, forward and backward, and uses a visible part of
    them (they are not vacuous)."""
    from tests import mlp_bounds as mb
    p, x, t, scale, mu, sd = _bounds_case(dims, n, 11)
    ref = mlp.predict(p, dims, x, scale, mu, sd)
    E = mb.forward_bounds(p, dims, x, scale, mu, sd)
    r = np.abs(mb.emulate_forward(p, dims, x, scale, mu, sd).astype(np.float64) - ref) / E
    assert np.all(r <= 0.75) and r.max() > 0.02, r.max()
    _, g = mlp.loss_and_grads(p, dims, x, t, scale, mu, sd)
    Eg = mb.gradient_bounds(p, dims, x, t, scale, mu, sd)
    rg = np.abs(mb.emulate_grads(p, dims, x, t, scale, mu, sd) - g) / Eg
    assert np.all(rg <= 0.75) and rg.max() > 0.02, rg.max()


def test_bf16_tolerances_catch_plausible_kernel_mistakes():
    """A square hidden weight used transposed, or a bias added to the wrong
    column, breaks the element-wise forward tolerance; inputs paired with the
    wrong rows, or output-bias gradients in the wrong order, break the
    backward one."""
    from tests import mlp_bounds as mb
    dims = (8, 16, 2, 4)
    p, x, t, scale, mu, sd = _bounds_case(dims, 50, 12)
    E = mb.forward_bounds(p, dims, x, scale, mu, sd)
    ref = mlp.predict(p, dims, x, scale, mu, sd)
    off = 8 * 16 + 16
    bad = p.copy()
    bad[off:off + 256] = p[off:off + 256].reshape(16, 16).T.ravel()
    assert np.any(np.abs(mb.emulate_forward(bad, dims, x, scale, mu, sd) - ref) > E)
    bad = p.copy()
    bb = off + 256
    bad[bb:bb + 16] = np.roll(p[bb:bb + 16], 1)
    assert np.any(np.abs(mb.emulate_forward(bad, dims, x, scale, mu, sd) - ref) > E)
    _, g = mlp.loss_and_grads(p, dims, x, t, scale, mu, sd)
    Eg = mb.gradient_bounds(p, dims, x, t, scale, mu, sd)
    # inputs paired with the wrong targets (rows off by one)
    _, g_wrong = mlp.loss_and_grads(p, dims, np.roll(x, 1, axis=0), t, scale, mu, sd)
    assert np.any(np.abs(g_wrong - g) > Eg)
    # the bias gradient of the output layer left out of the flat vector order
    _, g_wrong = mlp.loss_and_grads(p, dims, x, t, scale, mu, sd)
    g_wrong[-4:] = np.roll(g_wrong[-4:], 1)
    assert np.any(np.abs(g_wrong - g) > Eg)
