"""FP64 CPU oracle of the surrogate MLP (test infrastructure, like the rest of
``oracle/``).  Plain definitions, written out in numpy:

    h_0 = x * in_scale
    z_l = h_{l-1} W_l + b_l,  h_l = GELU(z_l) = z_l Phi(z_l)     (l = 1..L)
    y   = h_L W_{L+1} + b_{L+1}
    L   = 1/(n d_out) sum_{m,j} (y_mj - (t_mj - mu_j)/sd_j)^2

and the chain rule for every parameter gradient.  Parameters are one flat
vector in the order W_1, b_1, ..., W_{L+1}, b_{L+1} (row-major W: input index
by output index).

The optimiser is Adam (Kingma and Ba, "Adam: A Method for Stochastic
Optimization", ICLR 2015, Algorithm 1) with bias-corrected first and second
moment estimates, element by element.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

SQRT1_2 = 1.0 / np.sqrt(2.0)
INV_SQRT_2PI = 1.0 / np.sqrt(2.0 * np.pi)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z * SQRT1_2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z * SQRT1_2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def layer_dims(d_in, h, L, d_out):
    return [(d_in if l == 0 else h, d_out if l == L else h) for l in range(L + 1)]


def n_params(d_in, h, L, d_out):
    return sum(K * N + N for K, N in layer_dims(d_in, h, L, d_out))


def unpack(params, d_in, h, L, d_out):
    out, off = [], 0
    p = np.asarray(params, dtype=np.float64)
    for K, N in layer_dims(d_in, h, L, d_out):
        W = p[off:off + K * N].reshape(K, N)
        off += K * N
        b = p[off:off + N]
        off += N
        out.append((W, b))
    return out


def forward(params, dims, x, in_scale=None):
    """Standardised output y and the cache for the backward pass."""
    d_in, h, L, d_out = dims
    layers = unpack(params, *dims)
    x = np.asarray(x, dtype=np.float64)
    hcur = x * (np.ones(d_in) if in_scale is None else np.asarray(in_scale, dtype=np.float64))
    hs, zs = [hcur], []
    for l, (W, b) in enumerate(layers):
        z = hcur @ W + b
        if l < L:
            zs.append(z)
            hcur = gelu(z)
            hs.append(hcur)
        else:
            y = z
    return y, (hs, zs, layers)


def predict(params, dims, x, in_scale=None, out_mean=None, out_std=None):
    y, _ = forward(params, dims, x, in_scale)
    d_out = dims[3]
    mu = np.zeros(d_out) if out_mean is None else np.asarray(out_mean, dtype=np.float64)
    sd = np.ones(d_out) if out_std is None else np.asarray(out_std, dtype=np.float64)
    return y * sd + mu


def loss_and_grads(params, dims, x, t, in_scale=None, out_mean=None, out_std=None):
    d_in, h, L, d_out = dims
    y, (hs, zs, layers) = forward(params, dims, x, in_scale)
    n = y.shape[0]
    mu = np.zeros(d_out) if out_mean is None else np.asarray(out_mean, dtype=np.float64)
    sd = np.ones(d_out) if out_std is None else np.asarray(out_std, dtype=np.float64)
    r = y - (np.asarray(t, dtype=np.float64) - mu) / sd
    loss = float((r * r).sum() / (n * d_out))
    dz = 2.0 * r / (n * d_out)
    grads = [None] * (L + 1)
    for l in range(L, -1, -1):
        W, b = layers[l]
        gW = hs[l].T @ dz
        gb = dz.sum(axis=0)
        grads[l] = (gW, gb)
        if l > 0:
            dz = (dz @ W.T) * gelu_grad(zs[l - 1])
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def init_params(dims, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for K, N in layer_dims(*dims):
        parts.append(rng.standard_normal(K * N) / np.sqrt(K))
        parts.append(np.zeros(N))
    return np.concatenate(parts)


def adam_update(params, grad, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba 2015, Algorithm 1), FP64, element-wise.

    step is the 1-based index t of this update; m1, m2 are the moment
    estimates after step t - 1 (zeros before the first step).  Returns the new
    (params, m1, m2):
        m1 <- beta1 m1 + (1 - beta1) g
        m2 <- beta2 m2 + (1 - beta2) g^2
        m1_hat = m1 / (1 - beta1^t),  m2_hat = m2 / (1 - beta2^t)
        params <- params - lr m1_hat / (sqrt(m2_hat) + eps)
    """
    g = np.asarray(grad, dtype=np.float64)
    m1 = beta1 * np.asarray(m1, dtype=np.float64) + (1.0 - beta1) * g
    m2 = beta2 * np.asarray(m2, dtype=np.float64) + (1.0 - beta2) * g * g
    m1_hat = m1 / (1.0 - beta1 ** step)
    m2_hat = m2 / (1.0 - beta2 ** step)
    new = np.asarray(params, dtype=np.float64) - lr * m1_hat / (np.sqrt(m2_hat) + eps)
    return new, m1, m2
