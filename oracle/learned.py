"""Learned projection for the FlyHash codes (test infrastructure).

The paper hashes with a learned projection (BioHash) before the
winner-take-all step, and trains it with a rule it does not spell out.
This module defines the learned form used here, in float64:

  projection   y = W2 relu(W1 x + b1) + b2      (d -> H -> L)
  code         the wta_k largest outputs of y, ties to the lower index
               (Def. 7's winner-take-all applied to y)
  inference    as the GPU computes it: x, W1, relu(...) and W2 rounded to
               bfloat16 before each product (float32 accumulation on the
               GPU), y rounded to bfloat16 before the winner-take-all
  training     the gradients by the chain rule, in float64 or, to compare
               with the GPU element by element, with every product operand
               rounded to bfloat16 where the GPU rounds it

Training objective (the paper gives none; this is the build's reading):
  soft code     c_j(x) = sigmoid((y_j - t(x)) / tau), t(x) the midpoint of
                the wta_k-th and (wta_k+1)-th largest y (held constant)
  soft sketch   S_j(V) = 1 - prod_{x in V} (1 - c_j(x))   (Def. 10's OR)
  soft Hamming  h(A, B) = sum_j S_j(A) + S_j(B) - 2 S_j(A) S_j(B)
  triplet loss  max(0, margin + h(Q, P) - h(Q, N)) for a query set Q, a
                set P among its exact top-10 by Hausdorff distance, and a
                random set N; averaged over the triplets of a batch.
"""
from __future__ import annotations

import numpy as np

from .lowp import bf16_bits, bf16_value


def bf16(x) -> np.ndarray:
    return bf16_value(bf16_bits(np.asarray(x, dtype=np.float32)))


def mlp(X, W1, b1, W2, b2, quantised: bool = False):
    """(pre-activation, hidden, output) of the projection, float64.  With
    quantised, operands are rounded to bfloat16 as on the GPU."""
    X = np.asarray(X, dtype=np.float64)
    if quantised:
        pre = bf16(X) @ bf16(W1).T + b1
        h = np.maximum(pre, 0.0)
        y = bf16(h) @ bf16(W2).T + b2
    else:
        pre = X @ W1.T + b1
        h = np.maximum(pre, 0.0)
        y = h @ W2.T + b2
    return pre, h, y


def wta_codes(Y, k: int) -> np.ndarray:
    """bool [n, L]: the k largest of each row, ties to the lower index."""
    Y = np.asarray(Y, dtype=np.float64)
    order = np.argsort(-Y, axis=1, kind="stable")[:, :k]
    out = np.zeros(Y.shape, dtype=bool)
    np.put_along_axis(out, order, True, axis=1)
    return out


def thresholds(Y, k: int) -> np.ndarray:
    """Midpoint of the k-th and (k+1)-th largest value of each row."""
    s = -np.sort(-np.asarray(Y, dtype=np.float64), axis=1)
    return 0.5 * (s[:, k - 1] + s[:, k])


def soft_codes(Y, k: int, tau: float, t=None):
    """Soft codes; t overrides the per-row thresholds (held constant)."""
    t = thresholds(Y, k) if t is None else np.asarray(t, dtype=np.float64)
    z = (np.asarray(Y, dtype=np.float64) - t[:, None]) / tau
    return 1.0 / (1.0 + np.exp(-z))


def soft_sketch(C) -> np.ndarray:
    return 1.0 - np.prod(1.0 - np.asarray(C, dtype=np.float64), axis=0)


def soft_hamming(Sa, Sb) -> float:
    return float(np.sum(Sa + Sb - 2.0 * Sa * Sb))


def set_thresholds(weights, sets, k: int):
    W1, b1, W2, b2 = weights
    return [thresholds(mlp(V, W1, b1, W2, b2)[2], k) for V in sets]


def triplet_loss(weights, sets, triplets, k: int, tau: float, margin: float, t_fixed=None) -> float:
    """Mean triplet loss; sets: list of [m_i, d] arrays; triplets: (q, p, n)
    indices; t_fixed: per-set thresholds to hold constant (default: computed)."""
    W1, b1, W2, b2 = weights
    S = []
    for i, V in enumerate(sets):
        _, _, y = mlp(V, W1, b1, W2, b2)
        S.append(soft_sketch(soft_codes(y, k, tau, None if t_fixed is None else t_fixed[i])))
    total = 0.0
    for q, p, n in triplets:
        total += max(0.0, margin + soft_hamming(S[q], S[p]) - soft_hamming(S[q], S[n]))
    return total / len(triplets)


def triplet_grads(weights, sets, triplets, k: int, tau: float, margin: float, quantised: bool = False,
                  trace: list | None = None):
    """Mean loss and its gradients (dW1, db1, dW2, db2), by the chain rule
    (thresholds held constant).

    quantised: the operands of every product are rounded to bfloat16 as on
    the GPU -- x, W1, relu(...) and W2 in the forward pass, and the output
    gradient dy and the pre-activation gradient dpre before the products
    that take them (dh = dy W2, dW2 = dy^T h, dW1 = dpre^T x); the bias
    gradients sum the unrounded dy and dpre.  trace (a list) receives, per
    set, the operands of those products and the soft quantities behind dy:
    (x, pre, h, dy, dy_q, dpre, dpre_q, W2_q, c, others, S) with the rounded
    ones as used (others: the product over the other members of 1 - c)."""
    W1, b1, W2, b2 = weights
    if quantised:
        rnd = bf16
    else:
        def rnd(a):
            return np.asarray(a, dtype=np.float64)
    W1q, W2q = rnd(W1), rnd(W2)
    fw = []
    for V in sets:
        Vq = rnd(V)
        pre = Vq @ W1q.T + b1
        hq = rnd(np.maximum(pre, 0.0))
        y = hq @ W2q.T + b2
        c = soft_codes(y, k, tau)
        fw.append((Vq, pre, hq, c, soft_sketch(c)))
    dS = [np.zeros_like(f[4]) for f in fw]
    loss = 0.0
    nt = len(triplets)
    for q, p, n in triplets:
        Sq, Sp, Sn = fw[q][4], fw[p][4], fw[n][4]
        l = margin + soft_hamming(Sq, Sp) - soft_hamming(Sq, Sn)
        if l > 0:
            loss += l
            dS[q] += (2.0 * (Sn - Sp)) / nt
            dS[p] += (1.0 - 2.0 * Sq) / nt
            dS[n] -= (1.0 - 2.0 * Sq) / nt
    loss /= nt
    gW1 = np.zeros_like(W1)
    gb1 = np.zeros_like(b1)
    gW2 = np.zeros_like(W2)
    gb2 = np.zeros_like(b2)
    for (V, pre, h, c, S), g in zip(fw, dS):
        # dS_j / dc_j(x) = prod over the other members of (1 - c_j)
        one_minus = 1.0 - c
        others = np.empty_like(c)
        for i in range(c.shape[0]):
            others[i] = np.prod(np.delete(one_minus, i, axis=0), axis=0)
        dc = g[None, :] * others
        dy = dc * c * (1.0 - c) / tau
        dyq = rnd(dy)
        gW2 += dyq.T @ h
        gb2 += dy.sum(axis=0)
        dh = dyq @ W2q
        dpre = dh * (pre > 0)
        dpreq = rnd(dpre)
        gW1 += dpreq.T @ V
        gb1 += dpre.sum(axis=0)
        if trace is not None:
            trace.append((V, pre, h, dy, dyq, dpre, dpreq, W2q, c, others, S))
    return loss, (gW1, gb1, gW2, gb2)
