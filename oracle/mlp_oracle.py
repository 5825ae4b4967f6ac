"""FP64 reference of the per-branch drag surrogate network.

TEST INFRASTRUCTURE ONLY (imported by the tests, the smoke check and the
benchmark's CPU leg; the product library never loads it).

The surrogate replaces the branch-wise drag-coefficient lookup of the analytic
model (paper Sec. 2.4, Eq. (2)) with a network trained on per-branch
momentum-exchange forces from the LBM.  The network maps 5 standardised
features (log10 Re_D, inclination alpha, generation, inflow intensity I_u,
midpoint height / H) through two hidden layers of 64 ReLU units to one output,
the branch force coefficient y = F_x / ((rho U^2 / 2) L D).

Parameters are packed in this order, 4609 values in all:
W1 (64 x 5, row-major, out x in), b1 (64), W2 (64 x 64), b2 (64), w3 (64),
b3 (1).

Precision of the GPU form:
- weights are stored in BF16, rounded to nearest even from an FP32 master
  copy; biases stay FP32; accumulation is FP32;
- the training form keeps activations in FP32;
- the inference form, which feeds matrix cores, also rounds each layer's input
  (scaled features, hidden activations) to BF16.
The oracle computes in FP64 with exactly those roundings applied.  Gradients
with respect to the master weights pass straight through the rounding.

Loss: mean over the batch of (y - t)^2 on the standardised target
(t = (y_target - y_mean) / y_std).  Optimiser: Adam (Kingma and Ba 2015) with
bias correction.
"""
import math

import numpy as np

N_IN, N_H = 5, 64
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("w3", (N_H,)), ("b3", (1,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SIZES)


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), via the FP32 bit pattern."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def _weights(p, weights_bf16):
    w = unpack(p)
    if weights_bf16:
        for k in ("W1", "W2", "w3"):
            w[k] = bf16_round(w[k])
    return w


def forward(p, X, scale=None, weights_bf16=True, act_bf16=False):
    """Network output (standardised units) for rows X (n, 5) of raw features.
    scale = (x_mean, x_std) or None.  Returns (y, cache)."""
    w = _weights(p, weights_bf16)
    x = np.asarray(X, dtype=np.float64)
    if scale is not None:
        x = (x - np.asarray(scale[0])) / np.asarray(scale[1])
    rnd = bf16_round if act_bf16 else (lambda a: a)
    x0 = rnd(x)
    z1 = x0 @ w["W1"].T + w["b1"]
    h1 = rnd(np.maximum(z1, 0.0))
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["w3"] + w["b3"][0]
    return y, (w, x0, z1, h1, z2, h2)


def loss_grad(p, X, T, scale=None, weights_bf16=True):
    """Mean-square loss and its gradient (4609) for targets T (standardised)."""
    y, (w, x0, z1, h1, z2, h2) = forward(p, X, scale, weights_bf16, act_bf16=False)
    n = len(y)
    r = y - np.asarray(T, dtype=np.float64)
    loss = np.mean(r * r)
    dy = 2.0 * r / n
    g = {"b3": np.array([dy.sum()]), "w3": h2.T @ dy}
    dz2 = np.outer(dy, w["w3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ w["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ x0
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def tree_cd_sweep(p, scale, yscale, feat_fixed, lgd, w, re_h, intensity, lo, hi, area, cylinder_cd):
    """Surrogate C_D of one tree at each Re_H (inference form): for each branch
    the features (log10 Re_D clamped to [log10 lo, log10 hi], alpha,
    generation, I_u, midpoint height / H), the network output in target units,
    scaled by C_d(Re_D) / C_d(Re_D,clamped) outside the range; then
    sum_b y_b w_b / area.  feat_fixed: (n, 3) alpha, generation, height;
    lgd: log10(D / H); w: L D / H^2."""
    out = []
    for r in np.atleast_1d(re_h):
        lre = math.log10(r) + lgd
        lc = np.clip(lre, math.log10(lo), math.log10(hi))
        X = np.column_stack([lc, feat_fixed[:, 0], feat_fixed[:, 1], np.full(len(lgd), intensity), feat_fixed[:, 2]])
        y, _ = forward(p, X, scale=scale, weights_bf16=True, act_bf16=True)
        y = y * yscale[1] + yscale[0]
        y = y * cylinder_cd(10.0 ** lre, intensity) / cylinder_cd(10.0 ** lc, intensity)
        out.append(np.sum(y * w) / area)
    return np.array(out)
