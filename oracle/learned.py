"""Learned first-round sample counts (oracle; test infrastructure only).

Not a method of the paper: a predictor that plugs into the adaptive range
finder of Sec. 3.3.  For every sibling pair (t1, t2) = (2p, 2p+1) of level l
it predicts log(1 + c), c the number of sample columns the pair held when
the Halko-Martinsson-Tropp estimator accepted its basis in a plain adaptive
build (all its columns if it never did); the level's first sampling round
then takes max_p (predicted c_p) + oversample columns at once, and the
estimator of the plain method still decides when sampling stops (extra
rounds of rank_cap + oversample columns when the prediction fell short).

Features of pair p at level l (16 values):
  0   l / L
  1   log2 |t2| / 16
  2-4 extents of the bounding box of t2, largest first, divided by the
      largest extent of the root box (missing dimensions: 0)
  5   log10 of the aspect ratio (largest + d) / (smallest + d) of that box
      over its dimensions, d = 1e-12 times the root extent, divided by 4
  6   dimension / 3
  7   log10(eps) / 10, eps the relative construction tolerance
  8-14 for i = 2, 4, 8, 16, 32, 64, 128: max(log10(sigma_i / sigma_1), -16) / 16
      over the singular values of B0 of the parent pair (level l - 1, pair
      p // 2), -1 where the parent has fewer than i values or sigma_1 = 0;
      0 at level 1 (no parent)
  15  log2(1 + parent rank) / 10; -1 at level 1

Network: 16 -> 64 -> 64 -> 1 with ReLU after the two hidden layers.  The
products use the weights rounded to BF16 (round to nearest even from FP32);
inputs, activations and sums are exact here (FP64) and FP32 on the GPU.
Loss: mean over the batch of (y - target)^2.  Optimiser: Adam on FP32 master
weights (Kingma & Ba 2015, with bias correction).
"""
import math

import numpy as np

NFEAT = 16
HID = 64
SIG_IDX = (2, 4, 8, 16, 32, 64, 128)
PARAMS = ("W1", "b1", "W2", "b2", "W3", "b3")


def bf16_round(a):
    """FP64 array -> values representable in BF16 (via FP32, round to nearest even)."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def pair_features(tree, l, p, tol, parent_sig, parent_k):
    """The 16 features of sibling pair p at level l (see the module text)."""
    L = tree.L
    c2 = 2 * p + 1
    size = tree.size(l, c2)
    ext = np.sort(tree.hi[l][c2] - tree.lo[l][c2])[::-1]
    root_ext = float(np.max(tree.hi[0][0] - tree.lo[0][0]))
    root_ext = root_ext if root_ext > 0 else 1.0
    f = np.zeros(NFEAT)
    f[0] = l / L
    f[1] = math.log2(size) / 16.0
    for d in range(min(3, len(ext))):
        f[2 + d] = ext[d] / root_ext
    dd = 1e-12 * root_ext
    f[5] = math.log10((ext[0] + dd) / (ext[-1] + dd)) / 4.0 if len(ext) > 1 else 0.0
    f[6] = tree.dim / 3.0
    f[7] = math.log10(tol) / 10.0
    if l == 1:
        f[15] = -1.0
        return f
    s = np.asarray(parent_sig, dtype=np.float64)
    for q, i in enumerate(SIG_IDX):
        if len(s) >= i and s[0] > 0:
            r = s[i - 1] / s[0]
            f[8 + q] = max(math.log10(r), -16.0) / 16.0 if r > 0 else -1.0
        else:
            f[8 + q] = -1.0
    f[15] = math.log2(1 + parent_k) / 10.0
    return f


def level_features(tree, pr, l, tol):
    """Features of every pair of level l from a finished peel (PeelResult)."""
    out = []
    for p in range(1 << (l - 1)):
        if l == 1:
            out.append(pair_features(tree, l, p, tol, [], 0))
        else:
            q = p // 2
            out.append(pair_features(tree, l, p, tol, pr.sig[l - 1][q], int(pr.kw[l - 1][q])))
    return np.array(out)


def init_weights(seed):
    """He-normal initial weights (FP32), zero biases."""
    g = np.random.Generator(np.random.PCG64(seed))
    W = {
        "W1": g.standard_normal((HID, NFEAT)) * math.sqrt(2.0 / NFEAT),
        "b1": np.zeros(HID),
        "W2": g.standard_normal((HID, HID)) * math.sqrt(2.0 / HID),
        "b2": np.zeros(HID),
        "W3": g.standard_normal((1, HID)) * math.sqrt(2.0 / HID),
        "b3": np.zeros(1),
    }
    return {k: v.astype(np.float32) for k, v in W.items()}


def _eff(W, round_weights):
    return {k: (bf16_round(v) if round_weights and k.startswith("W") else v.astype(np.float64))
            for k, v in W.items()}


def forward(W, X, round_weights=True):
    """y (batch,) and the activations needed by backward."""
    E = _eff(W, round_weights)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ E["W1"].T + E["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ E["W2"].T + E["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ E["W3"][0] + E["b3"][0]
    return y, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2, E=E)


def backward(cache, y, target):
    """Loss and gradients of the mean squared error with respect to every
    parameter (the products use the same rounded weights as the forward)."""
    X, h1, h2, E = cache["X"], cache["h1"], cache["h2"], cache["E"]
    B = X.shape[0]
    d = y - np.asarray(target, dtype=np.float64)
    loss = float(np.mean(d * d))
    dy = 2.0 * d / B
    g = {}
    g["W3"] = (dy @ h2)[None, :]
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, E["W3"][0]) * (cache["z2"] > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ E["W2"]) * (cache["z1"] > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return loss, g


def adam_step(W, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the FP32 master weights (t = step number, from 1)."""
    Wn, mn, vn = {}, {}, {}
    for k in PARAMS:
        mk = beta1 * m[k].astype(np.float64) + (1 - beta1) * g[k]
        vk = beta2 * v[k].astype(np.float64) + (1 - beta2) * g[k] * g[k]
        mh = mk / (1 - beta1 ** t)
        vh = vk / (1 - beta2 ** t)
        Wn[k] = (W[k].astype(np.float64) - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
        mn[k] = mk.astype(np.float32)
        vn[k] = vk.astype(np.float32)
    return Wn, mn, vn


def first_round_width(pred_log1p_cols, oversample, base, limit=1024):
    """Level width from the per-pair predictions: max_p (exp(y_p) - 1), rounded
    up, plus oversample; never below the plain width `base`, at most limit - base."""
    if len(pred_log1p_cols) == 0:
        return base
    k = max(0.0, math.expm1(float(np.max(pred_log1p_cols))))
    return int(min(max(base, math.ceil(k) + oversample), limit - base))
