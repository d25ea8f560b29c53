"""The two filter layers of the cascade search (Alg. 6, filtering steps).

Query side (first steps of Alg. 6): the query's count Bloom filter C_Q
and its sketch S_Q are built from the query codes exactly as for a
database set (Algs. 3 and 5).  The positions P are the first A entries of
an argsort of C_Q in descending order; equal counts keep ascending
position order.

First layer (inverted index): set j enters F1 when some p in P has
C^(j)[p] >= M.  F1 is a set, so walking the sorted inverted lists of
Def. 9 or testing every set directly gives the same F1; this module uses
the direct test and `oracle.index` holds the literal list walk.

Second layer (sketches): every set of F1 is scored by the Hamming
distance between S_Q and S^(j), and the T smallest are kept.  The heap of
Alg. 6 stores (d, i) pairs and replaces only on a strictly smaller d; run
over F1 in ascending id order that keeps the first T sets of F1 ordered
by (distance, id), which is what `second_filter` returns.  The heap's
capacity c and the test against T are read as one parameter, T.
"""
from __future__ import annotations

import numpy as np


def query_sketches(HQ: np.ndarray):
    """C_Q (int64 [L]) and S_Q (bool [L]) from the query codes [m_q, L]."""
    HQ = np.asarray(HQ, dtype=bool)
    return HQ.sum(axis=0).astype(np.int64), HQ.any(axis=0)


def top_positions(C_Q: np.ndarray, A: int) -> np.ndarray:
    """First A positions of argsort-descending(C_Q); ties to lower position."""
    pos = np.arange(len(C_Q))
    order = np.lexsort((pos, -np.asarray(C_Q, dtype=np.int64)))
    return order[:A]


def first_filter(C: np.ndarray, P: np.ndarray, M: int) -> np.ndarray:
    """bool [n]: membership of each set in F1."""
    return (np.asarray(C)[:, P] >= M).any(axis=1)


def hamming(S_Q: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Hamming distance between the query sketch and every set sketch."""
    return np.count_nonzero(np.asarray(B, dtype=bool) != np.asarray(S_Q, dtype=bool)[None, :],
                            axis=1).astype(np.int64)


def second_filter(member: np.ndarray, scores: np.ndarray, T: int):
    """F2 ids and their scores: first min(T, |F1|) of F1 by (score, id)."""
    ids = np.flatnonzero(member)
    order = np.lexsort((ids, scores[ids]))
    keep = ids[order][:T]
    return keep, scores[keep]
