"""Second, independently written FP64 spin-image reference (vectorised NumPy).

TEST INFRASTRUCTURE ONLY.  It restates Section 2.1, Algorithm 1 with whole
arrays instead of loops and has no boundary flags; it exists to cross-check
the C oracle on tiny scenes (M up to a few hundred), where both must agree to
rounding.  Same readings as the C oracle: angle test as c >= cos S (vacuous for
S >= pi), row coordinate v = W/2 - beta/B, column u = alpha/B, self-pair
included, ceil binning counted when 0 <= k, l < W, bilinear counted when the
2x2 footprint is inside (0 <= v < W-1, u < W-1).
"""
from __future__ import annotations

import math

import numpy as np


def spin_images(xyz, nrm, idx, W, bin, support_angle, mode=0):
    X = np.asarray(xyz, dtype=np.float32).astype(np.float64)
    Nn = np.asarray(nrm, dtype=np.float32).astype(np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    B = float(np.float32(bin))
    S = float(np.float32(support_angle))
    P = X[idx]                       # (N, 3)
    Np = Nn[idx]
    D = X[None, :, :] - P[:, None, :]            # (N, M, 3)
    beta = np.einsum("nk,nmk->nm", Np, D)
    alpha = np.sqrt(np.clip(np.einsum("nmk,nmk->nm", D, D) - beta ** 2, 0.0, None))
    cosang = Np @ Nn.T                            # (N, M)
    ok = np.ones_like(beta, dtype=bool) if S >= math.pi else cosang >= math.cos(S)
    v = W / 2.0 - beta / B
    u = alpha / B
    n_img = len(idx)
    img = np.zeros((n_img, W, W))
    rows = np.repeat(np.arange(n_img), X.shape[0]).reshape(n_img, -1)
    if mode == 1:
        k = np.ceil(v)
        l = np.ceil(u)
        inside = ok & (k >= 0) & (k < W) & (l >= 0) & (l < W)
        np.add.at(img, (rows[inside], k[inside].astype(int), l[inside].astype(int)), 1.0)
    else:
        inside = ok & (v >= 0) & (v < W - 1) & (u < W - 1)
        fi, fj = np.floor(v), np.floor(u)
        a, b = v - fi, u - fj
        r, i0, j0 = rows[inside], fi[inside].astype(int), fj[inside].astype(int)
        aa, bb = a[inside], b[inside]
        np.add.at(img, (r, i0, j0), (1 - aa) * (1 - bb))
        np.add.at(img, (r, i0 + 1, j0), aa * (1 - bb))
        np.add.at(img, (r, i0, j0 + 1), (1 - aa) * bb)
        np.add.at(img, (r, i0 + 1, j0 + 1), aa * bb)
    return img, inside.sum(axis=1).astype(np.int64)
