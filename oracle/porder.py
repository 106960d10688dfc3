"""Oracle for the per-pair truncation order (TEST INFRASTRUCTURE ONLY: only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import
this module).  Plain numpy in FP64 unless stated; shares nothing with the HIP
library.

The method fixes one order p for all M2L interactions (Sec. 2, p ~
log(TOL)/log(theta)).  The learned variant predicts an order per weak pair
(T, S) from 8 features with an MLP 8 -> 32 -> 1 (ReLU), trained with the
pinball (quantile) loss on labels from high-order runs (see orc_labels in the
C oracle).  This module holds:

  features(tree, A, p)      the 8 features of every weak pair, FP64
  forward / loss / grad     the MLP and the pinball loss, FP64, by hand
  adam_step                 one bias-corrected Adam step (Kingma & Ba)
  orders(model, F, delta, p) the orders the evaluation uses, with the same
                            decision arithmetic as the library (FP32)

Feature definitions (schema 1), for target box T at level l of L and source
box S in weak(T), d = |c_T - c_S|, rho the box radii, sigma = max(rho, 2^-20
rho_root), ahat_k = a_k / sigma^k for k = 0..K, K = min(p, 20):
  f0 rho_S/d, f1 rho_T/d, f2 (rho_S+rho_T)/d, f3 l/L,
  f4 log10(|ahat_S|_1 / |ahat_root|_1),
  f5 log10(sum_{k>K/2} |ahat_{S,k}| / |ahat_S|_1),
  f6 log10(|ahat_S|_1 / sum_{S' in weak(T)} |ahat_S'|_1),
  f7 log10(|weak(T)|),
log10 arguments floored at 1e-300.

Model layout (353 floats): [W1 32x8][b1 32][W2 32][b2 1] (321 trainable),
then [mu 8][isd 8][lo 8][hi 8]; y = W2 . relu(W1 ((f - mu) isd) + b1) + b2.
Orders: clamp(ceil(y + delta), 4, p); a pair with a feature outside [lo, hi]
keeps p.
"""
from __future__ import annotations

import numpy as np

NFEAT, HID = 8, 32
NPARAM = HID * NFEAT + 2 * HID + 1          # 321
MODEL_FLOATS = NPARAM + 4 * NFEAT           # 353
FEAT_K = 20
QMIN = 4


def _box_offset(l):
    return (4 ** l - 1) // 3


def box_norms(A, radius, p):
    """n1 = sum_{k<=K} |a_k| / sigma^k and the part over k > K/2, per box."""
    K = min(p, FEAT_K)
    sig = np.maximum(radius, max(radius[0] * 2.0 ** -20, 1e-300))
    k = np.arange(K + 1)
    v = np.abs(A[:, :K + 1]) / sig[:, None] ** k[None, :]
    return v.sum(axis=1), v[:, 2 * k > K].sum(axis=1)


def features(tree, A, p):
    """[n_weak, 8] FP64 features in tree.weak_pairs() order."""
    lv, tb, sb = tree.weak_pairs()
    n1, tail = box_norms(A, tree.radius, p)
    gT = np.array([_box_offset(l) for l in lv], np.int64) + tb
    gS = np.array([_box_offset(l) for l in lv], np.int64) + sb
    d = np.maximum(np.abs(tree.centre[gT] - tree.centre[gS]), 1e-300)
    rS, rT = tree.radius[gS], tree.radius[gT]
    # share denominator and weak count per target box
    den = np.zeros(len(tree.radius))
    np.add.at(den, gT, n1[gS])
    nweak = np.zeros(len(tree.radius), np.int64)
    np.add.at(nweak, gT, 1)
    lg = lambda x: np.log10(np.maximum(x, 1e-300))
    F = np.empty((lv.size, NFEAT))
    F[:, 0] = rS / d
    F[:, 1] = rT / d
    F[:, 2] = (rS + rT) / d
    F[:, 3] = lv / tree.L if tree.L > 0 else 0.0
    F[:, 4] = lg(n1[gS] / max(n1[0], 1e-300))
    F[:, 5] = lg(tail[gS] / np.maximum(n1[gS], 1e-300))
    F[:, 6] = lg(n1[gS] / np.maximum(den[gT], 1e-300))
    F[:, 7] = np.log10(np.maximum(nweak[gT], 1))
    return F


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    W1 = w[o:o + HID * NFEAT].reshape(HID, NFEAT); o += HID * NFEAT
    b1 = w[o:o + HID]; o += HID
    W2 = w[o:o + HID]; o += HID
    b2 = w[o]; o += 1
    mu = w[o:o + NFEAT]; o += NFEAT
    isd = w[o:o + NFEAT]; o += NFEAT
    lo = w[o:o + NFEAT]; o += NFEAT
    hi = w[o:o + NFEAT]
    return W1, b1, W2, b2, mu, isd, lo, hi


def forward(w, F, want_hidden=False):
    """y = W2 . relu(W1 x + b1) + b2 with x = (f - mu) * isd, FP64."""
    W1, b1, W2, b2, mu, isd, _, _ = unpack(w)
    X = (np.asarray(F, np.float64) - mu) * isd
    Z = X @ W1.T + b1
    H = np.maximum(Z, 0.0)
    y = H @ W2 + b2
    return (y, X, Z, H) if want_hidden else y


def pinball(u, tau):
    """rho_tau(u) = u (tau - [u < 0])."""
    return u * (tau - (u < 0))


def loss(w, F, q, tau):
    return float(np.mean(pinball(np.asarray(q, np.float64) - forward(w, F), tau)))


def grad(w, F, q, tau):
    """Gradient of loss() over the 321 trainable parameters (back-propagation
    by hand).  At u = q - y = 0 the derivative of rho_tau is taken as tau, and
    relu'(0) as 0."""
    y, X, Z, H = forward(w, F, want_hidden=True)
    _, _, W2, _, _, _, _, _ = unpack(w)
    n = y.size
    u = np.asarray(q, np.float64) - y
    dy = -np.where(u >= 0, tau, tau - 1.0) / n      # d loss / d y
    dW2 = H.T @ dy
    db2 = dy.sum()
    dZ = np.outer(dy, W2) * (Z > 0)
    dW1 = dZ.T @ X
    db1 = dZ.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2, [db2]])


def adam_step(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step on the trainable part; returns new
    (w, m, v)."""
    w = np.array(w, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    w[:NPARAM] -= lr * mh / (np.sqrt(vh) + eps)
    return w, m, v


def orders(w, F, delta, p):
    """Per-pair orders as the evaluation takes them: the MLP in FP32 from FP32
    features, y + delta in FP32, ceil, clamp to [4, p]; p where a feature lies
    outside [lo, hi].  Also returns y + delta (FP32) for tie checks."""
    w32 = np.asarray(w, np.float32)
    W1, b1, W2, b2, mu, isd, lo, hi = (np.asarray(a, np.float32) for a in unpack(w32))
    F32 = np.asarray(F, np.float32)
    X = (F32 - mu) * isd
    Z = X @ W1.T + b1
    y = np.maximum(Z, np.float32(0)) @ W2 + np.float32(b2)
    yd = (y + np.float32(delta)).astype(np.float32)
    q = np.clip(np.ceil(np.clip(yd, -1e6, 1e6)), QMIN, p).astype(np.int64)
    inr = np.all((F32 >= lo) & (F32 <= hi), axis=1)
    q = np.where(inr, q, p)
    return q.astype(np.uint8), yd
