"""Element-wise tolerances for the surrogate MLP's BF16 kernels.

The GPU rounds every matrix operand to BF16 (unit roundoff u = 2^-9) and
accumulates in FP32; biases, pre-activations, GELU, the loss gradient and the
bias gradients stay in FP32.  Each entry of a product A B is a sum of terms
A_ik B_kj, and every rounding upstream of it -- of its own operands, and of
the activations and weights of earlier layers, which enter relative to the
same magnitudes -- perturbs it by a few u times its natural magnitude

    S_ij = sum_k |A_ik| |B_kj|     (outputs: out_std (|h_L| |W| + |b|);
                                    weight gradients: |h_{l-1}|^T |dZ_l|;
                                    bias gradients: sum over the batch |dZ_l|)

computed from the oracle's exact FP64 intermediates.  The tolerance of every
entry is 16 u S (3% of its natural magnitude) plus an FP32 floor; a gradient
entry's S also gets a quarter of its layer's mean S, since the errors that
reach it through the batch sum do not shrink with an accidentally small
|h| or |dZ| of its own row and column.  A numpy emulation of the kernels'
rounding sequence stays below 3/4 of these tolerances on the surrogate's
shapes for batches of 33 rows or more (tests/test_oracle_mlp.py; a single
row's loss gradient can be nearly all cancellation).  A misplaced or
mis-scaled term moves an entry by a sizeable part of S and fails it, whereas
a norm over a whole layer would hide a few wrong entries among hundreds of
thousands.  Only the oracle's intermediates enter; the GPU's values are
compared against them, never fed back.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp as orc_mlp

U16 = 2.0 ** -9    # BF16 unit roundoff
E32 = 2.0 ** -24   # FP32 unit roundoff
K_U = 16.0         # tolerance in units of u S
FLOOR = 0.25       # gradients: S plus this fraction of the layer's mean S


def forward_bounds(params, dims, x, in_scale, out_mean, out_std):
    """Element-wise tolerance of the physical output G~(x)."""
    y, (hs, zs, layers) = orc_mlp.forward(params, dims, x, in_scale)
    W, b = layers[-1]
    sd = np.asarray(out_std, dtype=np.float64)
    mu = np.asarray(out_mean, dtype=np.float64)
    S = sd * (np.abs(hs[-1]) @ np.abs(W) + np.abs(b))
    return K_U * U16 * S + 16 * E32 * (np.abs(y * sd) + np.abs(mu))


def gradient_bounds(params, dims, x, t, in_scale, out_mean, out_std):
    """Element-wise tolerance of the loss gradient (flat, logical order)."""
    d_in, h, L, d_out = dims
    y, (hs, zs, layers) = orc_mlp.forward(params, dims, x, in_scale)
    mu = np.asarray(out_mean, dtype=np.float64)
    sd = np.asarray(out_std, dtype=np.float64)
    n = y.shape[0]
    dz = 2.0 * (y - (np.asarray(t, dtype=np.float64) - mu) / sd) / (n * d_out)
    out = [None] * (L + 1)
    for l in range(L, -1, -1):
        W, b = layers[l]
        SW = np.abs(hs[l]).T @ np.abs(dz)
        Sb = np.abs(dz).sum(axis=0)
        out[l] = (K_U * U16 * (SW + FLOOR * SW.mean()), K_U * U16 * (Sb + FLOOR * Sb.mean()))
        if l > 0:
            dz = (dz @ W.T) * orc_mlp.gelu_grad(zs[l - 1])
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in out]) + 1e-30


def _round_bf16(a):
    """Round-to-nearest-even of FP32 values to BF16 (returned as FP32)."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    bits = a.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32)


def emulate_forward(params, dims, x, in_scale, out_mean, out_std):
    """The GPU's rounding sequence written out in numpy (BF16 operands, FP32
    products and sums, FP32 epilogues): a check that the tolerances above
    cover the arithmetic they model."""
    layers = orc_mlp.unpack(np.asarray(params, dtype=np.float32).astype(np.float64), *dims)
    L = dims[2]
    hcur = _round_bf16(np.asarray(x, np.float32) * np.asarray(in_scale, np.float32))
    for l, (W, b) in enumerate(layers):
        Wb = _round_bf16(W.astype(np.float32))
        z = (hcur.astype(np.float32) @ Wb.astype(np.float32)) + b.astype(np.float32)
        if l < L:
            hcur = _round_bf16(orc_mlp.gelu(z.astype(np.float64)).astype(np.float32))
        else:
            y = z
    return y.astype(np.float32) * np.asarray(out_std, np.float32) + np.asarray(out_mean, np.float32)


def emulate_grads(params, dims, x, t, in_scale, out_mean, out_std):
    """The backward pass with the GPU's roundings (numpy), flat logical order."""
    d_in, h, L, d_out = dims
    layers = orc_mlp.unpack(np.asarray(params, dtype=np.float32).astype(np.float64), *dims)
    Wb = [_round_bf16(W.astype(np.float32)) for W, _ in layers]
    H = [_round_bf16(np.asarray(x, np.float32) * np.asarray(in_scale, np.float32))]
    Z = []
    for l, (W, b) in enumerate(layers):
        z = H[l] @ Wb[l] + b.astype(np.float32)
        if l < L:
            Z.append(z)
            H.append(_round_bf16(orc_mlp.gelu(z.astype(np.float64)).astype(np.float32)))
        else:
            y = z
    n = y.shape[0]
    mu = np.asarray(out_mean, np.float32)
    sd = np.asarray(out_std, np.float32)
    r = y - (np.asarray(t, np.float32) - mu) / sd
    dz = np.float32(2.0 / (n * d_out)) * r
    out = [None] * (L + 1)
    for l in range(L, -1, -1):
        dzb = _round_bf16(dz)
        out[l] = (H[l].T @ dzb, dz.sum(axis=0))
        if l > 0:
            P = dzb @ Wb[l].T
            dz = (P * orc_mlp.gelu_grad(Z[l - 1].astype(np.float64)).astype(np.float32)).astype(np.float32)
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in out]).astype(np.float64)
