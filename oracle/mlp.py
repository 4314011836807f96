"""FP64 reference of the radiance-cache network.  TEST INFRASTRUCTURE ONLY.

The learned form replaces the recursion below bounce 2 by a small MLP
trained online on radiance computed by the full-depth tracer.  This module
states, step by step and in FP64, what the GPU network computes:

  encoding  x~ = 2 (x - lo) / (hi - lo) - 1 per axis (scene bounds lo, hi);
            for axis c in (x, y, z), frequency j in 0..5:
            feature[12 c + 2 j]     = sin(2^j pi x~_c)
            feature[12 c + 2 j + 1] = cos(2^j pi x~_c)
            features 36..38 = facing normal N_f, 39..41 = view direction V,
            42..63 = 0
  network   h_0 = bf16(features); h_l = bf16(relu(W_l h_{l-1})) for l = 1..5
            (W_l 64 x 64); y = W_6 h_5 (W_6 3 x 64); no biases.  Weights are
            the BF16 rounding of FP32 master weights.  The cache adds max(y, 0).
  loss      mean over samples and channels of (y - T)^2 / (sg(y)^2 + 0.01)
            (relative L2, sg = stop-gradient).
  backward  g_y = bf16(2 (y - T) / (y^2 + 0.01) / (3 N)); g_h5 = W_6^T g_y;
            g_z_l = bf16(g_h_l * [z_l > 0]); dW_l = g_z_l^T h_{l-1};
            g_h_{l-1} = W_l^T g_z_l; dW_6 = g_y^T h_5.  (Every operand of a
            product is BF16, as on the matrix cores; sums are FP64 here, FP32
            there.)
  Adam      m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
            w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
            on FP32 master weights (here FP64).

BF16 rounding is round-to-nearest-even to 8 significant bits.  With
rounding=False every step is plain FP64 (used for finite-difference pins).
"""
from __future__ import annotations

import numpy as np

WIDTH = 64
N_IN = 42
N_HIDDEN = 5
N_OUT = 3
N_FREQ = 6


def bf16_round(x):
    """Round to the nearest BF16 value (8 significant bits), ties to even."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)                     # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def encode(x, nf, v, lo, hi):
    """Features [N, 64] (FP64, before BF16 rounding) of hit points x with facing normals nf, view dirs v."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    xt = 2.0 * (x - lo) / (hi - lo) - 1.0
    f = np.zeros((len(x), WIDTH), np.float64)
    for c in range(3):
        for j in range(N_FREQ):
            a = (2.0 ** j) * np.pi * xt[:, c]
            f[:, 12 * c + 2 * j] = np.sin(a)
            f[:, 12 * c + 2 * j + 1] = np.cos(a)
    f[:, 36:39] = np.asarray(nf, np.float64).reshape(-1, 3)
    f[:, 39:42] = np.asarray(v, np.float64).reshape(-1, 3)
    return f


def _r(x, rounding):
    return bf16_round(x) if rounding else np.asarray(x, np.float64)


def forward(ws, feats, rounding=True):
    """Returns (y [N,3], cache) with cache = (h list, z list) for backward."""
    W = [_r(np.asarray(w, np.float64), rounding) for w in ws]
    h = [_r(feats, rounding)]
    zs = []
    for l in range(N_HIDDEN):
        z = h[-1] @ W[l].T
        zs.append(z)
        h.append(_r(np.maximum(z, 0.0), rounding))
    y = h[-1] @ W[N_HIDDEN].T
    return y, (W, h, zs)


def loss_and_grads(ws, feats, target, rounding=True):
    """Relative-L2 loss and gradients [dW_1 .. dW_6] (FP64) for one batch."""
    target = np.asarray(target, np.float64).reshape(-1, N_OUT)
    y, (W, h, zs) = forward(ws, feats, rounding)
    n = len(y)
    den = y * y + 0.01
    loss = float(np.mean((y - target) ** 2 / den))
    gy = _r(2.0 * (y - target) / den / (N_OUT * n), rounding)
    grads = [None] * (N_HIDDEN + 1)
    grads[N_HIDDEN] = gy.T @ h[N_HIDDEN]
    gh = gy @ W[N_HIDDEN]
    for l in range(N_HIDDEN - 1, -1, -1):
        gz = _r(gh * (zs[l] > 0.0), rounding)
        grads[l] = gz.T @ h[l]
        gh = gz @ W[l]
    return loss, grads, y


def adam_step(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step t >= 1) of master weights w; returns new (w, m, v)."""
    w = np.asarray(w, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def rel_mse(img, ref):
    """Relative MSE: mean over pixels and channels of (x - ref)^2 / (ref^2 + 0.01)."""
    img = np.asarray(img, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.mean((img - ref) ** 2 / (ref * ref + 0.01)))
