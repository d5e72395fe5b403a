"""fp64 reference of the learned block probe's training step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The probe is not part of the paper.  It is a 2-layer MLP, 5 inputs -> 64
ReLU units -> 1 logit, whose parameters are kept as 512 values in this
order: W1[64][5] (row = hidden unit), b1[64], w2[64], b2, zero padding.

Training objective: weighted binary cross-entropy on the logit z,

    loss_s = wt_s * (softplus(z_s) - y_s * z_s),

summed over the samples whose label y_s is 0 or 1 (label 255 = no sample).
The gradient is the plain chain rule of that sum through z = b2 + w2 . h,
h = relu(a), a = W1 f + b1.  With ``quantize_hidden`` the forward pass rounds
h exactly as inference does (bf16, 0 below 2^-8, 256 above 256) and the
backward pass treats that rounding as the identity where a > 0
(straight-through); without it the network is the smooth one, whose
gradient the finite-difference tests check.

Adam (Kingma and Ba, Algorithm 1) updates the fp32 master parameters from the
mean gradient (sum / number of samples).
"""
from __future__ import annotations

import numpy as np

H = 64
IN = 5
WORDS = 512
N_USED = H * IN + H + H + 1  # 449


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    W1 = p[:H * IN].reshape(H, IN)
    b1 = p[H * IN:H * IN + H]
    w2 = p[H * IN + H:H * IN + 2 * H]
    b2 = p[H * IN + 2 * H]
    return W1, b1, w2, b2


def pack(W1, b1, w2, b2):
    p = np.zeros(WORDS, dtype=np.float64)
    p[:H * IN] = np.asarray(W1, dtype=np.float64).reshape(-1)
    p[H * IN:H * IN + H] = b1
    p[H * IN + H:H * IN + 2 * H] = w2
    p[H * IN + 2 * H] = b2
    return p


def bf16_round(x):
    """Round to the nearest bf16 value, ties to even (x finite)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


def bf16_bits_to_float(b):
    b = np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def float_to_bf16_bits(x):
    """fp32 -> bf16 bit pattern, round to nearest even (finite inputs)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return (u >> 16).astype(np.uint16)


def sanitize(w):
    """Stored weight as the probe uses it: 0 for NaN or |w| < 2^-12,
    clamped to [-16, 16]."""
    w = np.asarray(w, dtype=np.float64).copy()
    w[np.isnan(w) | (np.abs(w) < 2.0 ** -12)] = 0.0
    return np.clip(w, -16.0, 16.0)


def quantize_hidden(a):
    a = np.asarray(a, dtype=np.float64)
    h = np.where(a > 0, bf16_round(np.where(a > 0, a, 1.0)), 0.0)
    h = np.where(h < 2.0 ** -8, 0.0, h)
    return np.minimum(h, 256.0)


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward_backward(params, feats, labels, weights, quantize=True):
    """Sum of the weighted BCE loss over valid samples, its gradient with
    respect to the 512 parameters, the sum of |per-sample contribution| of
    every gradient entry (the scale of its rounding error in any summation
    order), and the number of valid samples.

    params: 512 values (used as given); feats: [n, 5]; labels: [n] in
    {0, 1, 255}; weights: [n] sample weights."""
    W1, b1, w2, b2 = unpack(params)
    f = np.asarray(feats, dtype=np.float64)
    y = np.asarray(labels)
    valid = y != 255
    f, yv = f[valid], (y[valid] == 1).astype(np.float64)
    wt = np.asarray(weights, dtype=np.float64)[valid]
    a = f @ W1.T + b1                       # [n, 64]
    h = quantize_hidden(a) if quantize else np.maximum(a, 0.0)
    z = h @ w2 + b2                         # [n]
    loss = float(np.sum(wt * (softplus(z) - yv * z)))
    dz = wt * (sigmoid(z) - yv)             # dloss/dz
    act = (a > 0).astype(np.float64)
    dh = dz[:, None] * w2[None, :] * act    # dloss/da
    gW2 = dz @ h
    gb2 = dz.sum()
    gW1 = dh.T @ f
    gb1 = dh.sum(axis=0)
    g = pack(gW1, gb1, gW2, gb2)
    adz = np.abs(dz)
    adh = np.abs(dh)
    s = pack(adh.T @ np.abs(f), adh.sum(axis=0), adz @ np.abs(h), adz.sum())
    return loss, g, s, int(valid.sum())


def loss_only(params, feats, labels, weights, quantize=False):
    W1, b1, w2, b2 = unpack(params)
    f = np.asarray(feats, dtype=np.float64)
    y = np.asarray(labels)
    valid = y != 255
    f, yv = f[valid], (y[valid] == 1).astype(np.float64)
    wt = np.asarray(weights, dtype=np.float64)[valid]
    a = f @ W1.T + b1
    h = quantize_hidden(a) if quantize else np.maximum(a, 0.0)
    z = h @ w2 + b2
    return float(np.sum(wt * (softplus(z) - yv * z)))


def adam(master, m, v, grad_sum, count, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on the mean gradient; returns new (master, m, v)."""
    g = np.asarray(grad_sum, dtype=np.float64) / max(count, 1)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    master = np.asarray(master, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps)
    master[N_USED:] = 0.0
    return master, m, v
