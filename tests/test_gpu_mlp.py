"""GPU parity of the surrogate MLP's BF16 MFMA forward and backward kernels
against the FP64 oracle (oracle/mlp.py).

BF16 rounds every matrix operand to 8 significant bits (unit roundoff
u = 2^-9), with FP32 accumulation.  Each product therefore carries at most
about 2u of norm-wise relative error (one rounding per operand), and GELU's
slope stays within [-0.13, 1.13], so errors add up roughly linearly along the
chain of products: the forward output is allowed 2u per product (L + 1 of
them), a gradient 2u per product of the forward and backward chains
(2 (L + 1)).  The tests print the measured errors (typically 5e-3).
"""
import numpy as np
import pytest

from oracle import mlp as orc_mlp

pytestmark = pytest.mark.gpu

FULL = (168, 512, 3, 49)
TINY = (8, 16, 2, 4)
U_BF16 = 2.0 ** -9


def fwd_tol(dims):
    return 2 * U_BF16 * (dims[2] + 1)


def grad_tol(dims):
    return 2 * U_BF16 * 2 * (dims[2] + 1)


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


def _setup(pm, ctx, dims, n, seed):
    rng = np.random.default_rng(seed)
    p = orc_mlp.init_params(dims, seed) + 0.02 * rng.standard_normal(orc_mlp.n_params(*dims))
    x = rng.standard_normal((n, dims[0]))
    t = rng.standard_normal((n, dims[3]))
    scale = rng.uniform(0.5, 2.0, dims[0])
    mu, sd = rng.standard_normal(dims[3]), rng.uniform(0.5, 2.0, dims[3])
    net = pm.MLP(ctx, *dims, max_batch=max(n, 1), seed=1)
    net.set_params(p)
    net.set_io(scale, mu, sd)
    return net, p, x, t, scale, mu, sd


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dims,n", [(TINY, 7), (TINY, 130), (FULL, 1), (FULL, 300), (FULL, 1024)])
def test_forward_matches_oracle(pm, ctx, dims, n):
    net, p, x, t, scale, mu, sd = _setup(pm, ctx, dims, n, 3)
    y = net.forward(x).cpu().numpy()
    ref = orc_mlp.predict(p, dims, x, scale, mu, sd)
    err = _rel(y - mu, ref - mu)
    print("forward %s n=%d: relative error %.2e (bound %.2e)" % (dims, n, err, fwd_tol(dims)))
    assert err < fwd_tol(dims)
    net.close()


@pytest.mark.parametrize("dims,n", [(TINY, 33), (FULL, 256)])
def test_gradients_match_oracle(pm, ctx, dims, n):
    net, p, x, t, scale, mu, sd = _setup(pm, ctx, dims, n, 4)
    g = net.grads(x, t).astype(np.float64)
    _, ref = orc_mlp.loss_and_grads(p, dims, x, t, scale, mu, sd)
    off = 0
    for l, (K, N) in enumerate(orc_mlp.layer_dims(*dims)):
        for name, size in (("W", K * N), ("b", N)):
            e = _rel(g[off:off + size], ref[off:off + size])
            print("grad layer %d %s: relative error %.2e (bound %.2e)" % (l, name, e, grad_tol(dims)))
            assert e < grad_tol(dims)
            off += size
    net.close()


@pytest.mark.parametrize("dims,n", [(TINY, 7), (TINY, 130), (FULL, 1), (FULL, 300), (FULL, 1024)])
def test_forward_matches_oracle_elementwise(pm, ctx, dims, n):
    """Every output entry within its BF16 tolerance (16 u times the entry's
    natural magnitude, tests/mlp_bounds.py)."""
    from tests import mlp_bounds as mb
    net, p, x, t, scale, mu, sd = _setup(pm, ctx, dims, n, 5)
    y = net.forward(x).cpu().numpy().astype(np.float64)
    ref = orc_mlp.predict(p, dims, x, scale, mu, sd)
    tol = mb.forward_bounds(p, dims, x, scale, mu, sd)
    r = np.abs(y - ref) / tol
    print("forward %s n=%d: max error / tolerance %.3f" % (dims, n, r.max()))
    assert np.all(r <= 1.0), (np.unravel_index(np.argmax(r), r.shape), r.max())
    net.close()


@pytest.mark.parametrize("dims,n", [(TINY, 33), (FULL, 64), (FULL, 256)])
def test_gradients_match_oracle_elementwise(pm, ctx, dims, n):
    """Every gradient entry (all weights and biases) within its BF16
    tolerance (tests/mlp_bounds.py)."""
    from tests import mlp_bounds as mb
    net, p, x, t, scale, mu, sd = _setup(pm, ctx, dims, n, 6)
    g = net.grads(x, t).astype(np.float64)
    _, ref = orc_mlp.loss_and_grads(p, dims, x, t, scale, mu, sd)
    tol = mb.gradient_bounds(p, dims, x, t, scale, mu, sd)
    r = np.abs(g - ref) / tol
    print("gradients %s n=%d: max error / tolerance %.3f at entry %d" % (dims, n, r.max(), int(np.argmax(r))))
    assert np.all(r <= 1.0), (int(np.argmax(r)), r.max())
    net.close()


def test_adam_first_step_moves_each_weight_by_lr_against_its_gradient(pm, ctx):
    dims, n, lr = FULL, 256, 1e-3
    net, p, x, t, scale, mu, sd = _setup(pm, ctx, dims, n, 5)
    _, ref = orc_mlp.loss_and_grads(p, dims, x, t, scale, mu, sd)
    p0 = net.get_params().astype(np.float64)
    net.train_step(x, t, lr)
    d = net.get_params().astype(np.float64) - p0
    big = np.abs(ref) > 1e-2 * np.abs(ref).max()
    # first Adam step: m^ = g, v^ = g^2, so the step is lr * g / (|g| + eps) = lr * sign(g)
    agree = np.mean(np.sign(d[big]) == -np.sign(ref[big]))
    print("Adam step: sign agreement %.4f, |step|/lr median %.4f" % (agree, np.median(np.abs(d[big])) / lr))
    assert agree > 0.99
    assert abs(np.median(np.abs(d[big])) / lr - 1) < 0.01
    net.close()


def test_training_fits_a_teacher_network(pm, ctx):
    import torch
    dims = FULL
    rng = np.random.default_rng(8)
    teacher = orc_mlp.init_params(dims, 99)
    X = rng.standard_normal((8192, dims[0]))
    Y = orc_mlp.predict(teacher, dims, X)
    net = pm.MLP(ctx, *dims, max_batch=1024, seed=2)
    sd = Y.std(0)
    mu = Y.mean(0)
    net.set_io(None, mu, sd)
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    Yt = torch.tensor(Y, dtype=torch.float32, device="cuda")
    first = None
    for step in range(400):
        s = (step * 1024) % 8192
        loss = float(net.train_step(Xt[s:s + 1024], Yt[s:s + 1024], 1e-3).item())
        if first is None:
            first = loss
    print("teacher fit: loss %.4f -> %.4f" % (first, loss))
    assert loss < first / 5
    # the trained GPU network agrees with the oracle evaluated at its own weights
    Xv = rng.standard_normal((512, dims[0]))
    y = net.forward(Xv).cpu().numpy()
    ref = orc_mlp.predict(net.get_params().astype(np.float64), dims, Xv, None, mu, sd)
    assert _rel(y - mu, ref - mu) < fwd_tol(dims)
    net.close()


def test_adam_steps_match_the_fp64_oracle_elementwise(pm, ctx):
    """Six Adam steps (Kingma and Ba, Algorithm 1: bias-corrected moments,
    beta = (0.9, 0.999), eps = 1e-8) on one batch from identical weights.

    (a) Arithmetic.  The train step uses the gradient pm_mlp_grads returns at
    the same weights, so at every step the GPU's new weights must equal the
    FP64 oracle's Adam update applied to the GPU's own gradients (moments
    carried over the same gradient sequence), element by element, to FP32
    rounding.  The moment updates b m + (1 - b) g round relative to their
    terms, not their (possibly cancelling) result, so the bound is 2 ulp of
    the weight, plus lr c1 8 s 2^-24 S1 / (sqrt(v^) + eps) with S1 the same
    exponential average of |g| as m1 (t = s steps, c1 = 1 / (1 - b1^s)),
    plus 1e-5 of the update (division, square root, constants in FP32).

    (b) Trajectory.  Against the oracle's own FP64 run (FP64 gradients at its
    own weights), every parameter stays within the bound that the measured
    gradient differences dg_s = g_gpu,s - g_ref,s imply for Adam:
        |m^_gpu - m^_ref| <= sum_s w1_s |dg_s| / (1 - b1^t) = A_m,
        |sqrt(v^_gpu) - sqrt(v^_ref)| <= (sum_s w2_s dg_s^2 / (1 - b2^t))^(1/2) = A_v
    (the triangle inequality of the weighted 2-norm), so the update differs by
    at most (A_m + |u_ref| A_v) / (sqrt(v^_gpu) + eps), summed over steps
    with the learning rate; the gradient differences themselves are within
    the BF16 bound of test_gradients_match_oracle, layer by layer."""
    dims, n, lr, steps = FULL, 256, 1e-3, 6
    b1, b2, eps = 0.9, 0.999, 1e-8
    net, p, x, t, scale, mu, sd = _setup(pm, ctx, dims, n, 6)
    p0 = net.get_params().astype(np.float64)
    # (a) and the GPU's gradient sequence
    m1 = np.zeros_like(p0)
    m2 = np.zeros_like(p0)
    S1 = np.zeros_like(p0)
    g_gpu, p_gpu, tols = [], [p0], []
    worst_a = 0.0
    for s in range(1, steps + 1):
        g = net.grads(x, t).astype(np.float64)
        before = net.get_params().astype(np.float64)
        net.train_step(x, t, lr)
        after = net.get_params().astype(np.float64)
        ref, m1, m2 = orc_mlp.adam_update(before, g, m1, m2, s, lr, b1, b2, eps)
        S1 = b1 * S1 + (1 - b1) * np.abs(g)
        c1 = 1.0 / (1.0 - b1 ** s)
        vhat = m2 / (1.0 - b2 ** s)
        tol = (2 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
               + lr * c1 * 8 * s * 2.0 ** -24 * S1 / (np.sqrt(vhat) + eps)
               + 1e-5 * np.abs(ref - before) + 1e-30)
        r = np.abs(after - ref) / tol
        worst_a = max(worst_a, np.max(r))
        k = int(np.argmax(r))
        assert np.all(r <= 1), (s, k, before[k], after[k], ref[k], g[k], m1[k], m2[k], tol[k])
        tols.append(tol)
        g_gpu.append(g)
        p_gpu.append(after)
    # (b) the oracle's own FP64 run from the same start
    pr = p0.copy()
    r1 = np.zeros_like(pr)
    r2 = np.zeros_like(pr)
    bound = np.zeros_like(pr)
    dgs = []
    worst_g = 0.0
    for s in range(1, steps + 1):
        _, gr = orc_mlp.loss_and_grads(pr, dims, x, t, scale, mu, sd)
        # the measured gradient difference is within the BF16 bound, layer by layer
        off = 0
        for K, N in orc_mlp.layer_dims(*dims):
            for size in (K * N, N):
                e = _rel(g_gpu[s - 1][off:off + size], gr[off:off + size])
                worst_g = max(worst_g, e)
                assert e < grad_tol(dims)
                off += size
        dgs.append(g_gpu[s - 1] - gr)
        pr_new, r1, r2 = orc_mlp.adam_update(pr, gr, r1, r2, s, lr, b1, b2, eps)
        u_ref = (pr - pr_new) / lr
        w1 = np.array([(1 - b1) * b1 ** (s - q) for q in range(1, s + 1)])
        w2 = np.array([(1 - b2) * b2 ** (s - q) for q in range(1, s + 1)])
        A_m = sum(w * np.abs(dg) for w, dg in zip(w1, dgs)) / (1 - b1 ** s)
        A_v = np.sqrt(sum(w * dg * dg for w, dg in zip(w2, dgs)) / (1 - b2 ** s))
        v_gpu = sum(w * g * g for w, g in zip(w2, g_gpu[:s])) / (1 - b2 ** s)
        bound += lr * (A_m + np.abs(u_ref) * A_v) / (np.sqrt(v_gpu) + eps)
        pr = pr_new
        slack = bound + sum(tols[:s])  # plus the FP32 arithmetic of (a) at every step so far
        d = np.abs(p_gpu[s] - pr)
        assert np.all(d <= slack), (s, np.max(d / slack))
    moved = np.abs(pr - p0)
    print("Adam x%d: arithmetic max err/tol %.3f; gradient rel err max %.2e; trajectory |p_gpu - p_ref| "
          "max %.2e (median bound %.2e, median move %.2e)" % (steps, worst_a, worst_g, np.max(d), np.median(bound),
                                                          np.median(moved)))
    net.close()
