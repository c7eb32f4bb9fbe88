"""FP64 reference of the iteration-count predictor (test infrastructure only).

The network maps per-column features to the logarithm of the number of
Krylov iterations the column needs:
    x' = (x - mean) * inv_std
    h1 = relu(W1 x' + b1), h2 = relu(W2 h1 + b2), y = W3 . h2 + b3
trained by mean-squared error with Adam (Kingma and Ba 2015).  Parameters
are one flat vector (same layout as the GPU library):
    [0:5] mean, [5:10] inv_std, W1 (64x5, row-major), b1 (64),
    W2 (64x64), b2 (64), W3 (64), b3 (1)  -> 4619 values, the last 4609 trainable.

Features of column j (atom c, orbital o) on its local subspace L:
    f0 number of off-diagonal blocks of c's block row inside L
    f1 mean over those blocks of ||H_cb[o, :]||_2
    f2 max of the same
    f3 |H_jj - mean of H_ii over the orbitals i of L with i % 4 == o|
    f4 number of local orbitals.
"""
from __future__ import annotations

import numpy as np

NF, NH = 5, 64
OFF_W1 = 2 * NF
OFF_B1 = OFF_W1 + NH * NF
OFF_W2 = OFF_B1 + NH
OFF_B2 = OFF_W2 + NH * NH
OFF_W3 = OFF_B2 + NH
OFF_B3 = OFF_W3 + NH
NPARAM = OFF_B3 + 1


def unpack(p):
    return (p[0:NF], p[NF:2 * NF], p[OFF_W1:OFF_B1].reshape(NH, NF), p[OFF_B1:OFF_W2],
            p[OFF_W2:OFF_B2].reshape(NH, NH), p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def forward(p, x):
    """y[n] for features x[n, 5] (FP64)."""
    mean, istd, W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, np.float64))
    xs = (np.asarray(x, np.float64) - mean) * istd
    h1 = np.maximum(xs @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ W3 + b3


def loss_and_grad(p, x, t):
    """MSE loss (1/n) sum (y - t)^2 and its gradient over the whole vector
    (the normalisation entries get zero gradient)."""
    p = np.asarray(p, np.float64)
    mean, istd, W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, np.float64)
    t = np.asarray(t, np.float64)
    n = x.shape[0]
    xs = (x - mean) * istd
    a1 = xs @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ W3 + b3
    loss = np.mean((y - t) ** 2)
    dy = 2.0 * (y - t) / n
    g = np.zeros_like(p)
    g[OFF_W3:OFF_B3] = h2.T @ dy
    g[OFF_B3] = dy.sum()
    d2 = np.outer(dy, W3) * (a2 > 0)
    g[OFF_W2:OFF_B2] = (d2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = d2.sum(0)
    d1 = (d2 @ W2) * (a1 > 0)
    g[OFF_W1:OFF_B1] = (d1.T @ xs).ravel()
    g[OFF_B1:OFF_W2] = d1.sum(0)
    return loss, g


def adam_step(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of the trainable entries (step counts from 1)."""
    p, m, v = p.copy(), m.copy(), v.copy()
    sl = slice(OFF_W1, NPARAM)
    m[sl] = b1 * m[sl] + (1 - b1) * g[sl]
    v[sl] = b2 * v[sl] + (1 - b2) * g[sl] ** 2
    mh = m[sl] / (1 - b1 ** step)
    vh = v[sl] / (1 - b2 ** step)
    p[sl] = p[sl] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def features(bsr, loc_atoms, j):
    """Feature vector of column j on the local subspace given by loc_atoms (sorted)."""
    c, o = j // 4, j % 4
    loc = set(int(a) for a in loc_atoms)
    norms = []
    for t in range(bsr.row_ptr[c], bsr.row_ptr[c + 1]):
        b = int(bsr.col[t])
        if b == c or b not in loc:
            continue
        norms.append(np.linalg.norm(bsr.h[t][o, :]))
    diag = {}
    for a in loc_atoms:
        t = bsr.row_ptr[a] + int(np.nonzero(bsr.col[bsr.row_ptr[a]:bsr.row_ptr[a + 1]] == a)[0][0])
        diag[int(a)] = np.diag(bsr.h[t])
    same_type = np.array([diag[int(a)][o] for a in loc_atoms])
    f3 = abs(diag[c][o] - same_type.mean())
    nb = len(norms)
    return np.array([nb, np.mean(norms) if nb else 0.0, np.max(norms) if nb else 0.0, f3, 4 * len(loc_atoms)])
