"""FP64 reference of the per-image cost model -- TEST INFRASTRUCTURE ONLY.

The paper's earlier static split needed per-image timings measured on each
architecture (Section 2.3); the learned model predicts a per-image cost
instead.  This module is the plain definition used to check the library:

* ``features``: 12 numbers per oriented point from the point counts of the
  3 x 3 x 3 block of coarse cells around p (a coarse cell = s x s x s grid
  cells of edge h, s = 3, centred on p's cell) and from p's normal n:
    f0..f3  log1p of the count in the centre, the 6 face, 12 edge and 8
            corner neighbours;
    f4..f6  occupancy-weighted mean offset m = sum o(d) d / sum o;
    f7      m . n;
    f8      sum o(d) (d . n)^2 / sum o;
    f9      sum o(d) |d - (d . n) n|^2 / sum o;
    f10     log1p(sum o);
    f11     support radius / (s h).
  The grid is rebuilt here from the raw points exactly as the library
  defines it (origin = per-axis minimum, cell =
  floor((x - origin) / h) in float64, h = R_max (1 + 2e-5) / s).
* ``forward`` / ``backward``: MLP 12 -> 64 -> 64 -> 1 with ReLU, loss =
  mean((out - log1p(count))^2); analytic gradients.
* ``adam_step``: Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.

Parameter vector layout (5,057 values): W1 (64 x 12), b1 (64), W2 (64 x 64),
b2 (64), w3 (64), b3 (1), row-major.
"""
from __future__ import annotations

import numpy as np

SUB = 3
N_PARAMS = 64 * 12 + 64 + 64 * 64 + 64 + 64 + 1


def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = t[o:o + 768].reshape(64, 12); o += 768
    b1 = t[o:o + 64]; o += 64
    W2 = t[o:o + 4096].reshape(64, 64); o += 4096
    b2 = t[o:o + 64]; o += 64
    w3 = t[o:o + 64]; o += 64
    b3 = t[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def forward(theta, X):
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ w3 + b3
    return out, (X, z1, h1, z2, h2)


def loss_and_grad(theta, X, counts):
    """Mean squared error against log1p(counts) and its gradient (analytic)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    y = np.log1p(np.asarray(counts, dtype=np.float64))
    out, (X, z1, h1, z2, h2) = forward(theta, X)
    n = len(y)
    r = out - y
    loss = float(np.mean(r * r))
    dout = 2.0 * r / n
    gw3 = h2.T @ dout
    gb3 = dout.sum()
    dz2 = np.outer(dout, w3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gw3, gb3)


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def grid(xyz, max_support_radius):
    """(origin, h, dims, cell index per point) of the library's grid."""
    X = np.asarray(xyz, dtype=np.float32)
    lo = X.min(axis=0).astype(np.float64)
    ext = X.max(axis=0).astype(np.float64) - lo
    h = float(max_support_radius) * (1.0 + 2e-5) / SUB
    dims = (np.floor(ext / h) + 1).astype(np.int64)
    cell = np.floor((X.astype(np.float64) - lo) / h).astype(np.int64)
    return lo, h, dims, cell


def features(xyz, nrm, idx, max_support_radius, support_radius):
    lo, h, dims, cell = grid(xyz, max_support_radius)
    lin = (cell[:, 2] * dims[1] + cell[:, 1]) * dims[0] + cell[:, 0]
    occ = np.bincount(lin, minlength=int(np.prod(dims))).reshape(dims[2], dims[1], dims[0])
    # prefix sums to count any box of cells
    P = np.zeros((dims[2] + 1, dims[1] + 1, dims[0] + 1), dtype=np.int64)
    P[1:, 1:, 1:] = occ.cumsum(0).cumsum(1).cumsum(2)

    def box(z0, z1, y0, y1, x0, x1):
        z0, y0, x0 = max(z0, 0), max(y0, 0), max(x0, 0)
        z1, y1, x1 = min(z1, dims[2] - 1), min(y1, dims[1] - 1), min(x1, dims[0] - 1)
        if z1 < z0 or y1 < y0 or x1 < x0:
            return 0
        z1, y1, x1 = z1 + 1, y1 + 1, x1 + 1
        return int(P[z1, y1, x1] - P[z0, y1, x1] - P[z1, y0, x1] - P[z1, y1, x0]
                   + P[z0, y0, x1] + P[z0, y1, x0] + P[z1, y0, x0] - P[z0, y0, x0])

    N = np.asarray(nrm, dtype=np.float32).astype(np.float64)
    out = np.zeros((len(idx), 12))
    half = SUB // 2
    for r, i in enumerate(idx):
        cx, cy, cz = cell[i]
        n = N[i]
        o = {}
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    o[(dx, dy, dz)] = box(cz + SUB * dz - half, cz + SUB * dz + half,
                                          cy + SUB * dy - half, cy + SUB * dy + half,
                                          cx + SUB * dx - half, cx + SUB * dx + half)
        tot = sum(o.values())
        shells = [0, 0, 0, 0]
        m = np.zeros(3)
        s8 = s9 = 0.0
        for d, c in o.items():
            shells[sum(abs(t) for t in d)] += c
            dv = np.array(d, dtype=np.float64)
            m += c * dv
            dn = dv @ n
            s8 += c * dn * dn
            s9 += c * float(np.sum((dv - dn * n) ** 2))
        m /= tot
        out[r, 0:4] = np.log1p(shells)
        out[r, 4:7] = m
        out[r, 7] = m @ n
        out[r, 8] = s8 / tot
        out[r, 9] = s9 / tot
        out[r, 10] = np.log1p(tot)
        out[r, 11] = support_radius / (SUB * h)
    return out, occ
