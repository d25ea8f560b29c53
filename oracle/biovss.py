"""The full-scan search of the paper's first method (Alg. 2, Sec. 4.1.2).

Test infrastructure (see the package docstring): only tests, the smoke
check and the benchmark's CPU baseline may use it.

Alg. 2 encodes the query's vectors with the same FlyHash as the database
(Def. 7), measures every database set by a Hausdorff distance over binary
codes -- Def. 4 with the Hamming distance between codes in place of the
Euclidean distance -- keeps the c sets of smallest such distance, measures
those by the exact Hausdorff distance and returns the k nearest.

hamming_matrix     Hamming distances between two sets of codes
hamming_hausdorff  Haus^H: Def. 4 applied to that matrix
full_scores        Haus^H of the query codes to every database set
full_candidates    the first c sets by (Haus^H, id)
search_full        the whole of Alg. 2: candidates, then the first k by
                   (exact squared Hausdorff distance, id)

Readings: the candidate set keeps every set with Haus^H at most the c-th
smallest; here exactly min(c, n) sets are kept, ties to the lower id (the
same reading as the top-T of Alg. 6), and likewise exactly min(k, c) results.
"""
from __future__ import annotations

import numpy as np

from .flyhash import codes
from .hausdorff import hausdorff_from_matrix, hausdorff_sq


def hamming_matrix(HA, HB) -> np.ndarray:
    """[|A|, |B|] number of positions where code a_i and code b_j differ."""
    HA = np.asarray(HA, dtype=bool)
    HB = np.asarray(HB, dtype=bool)
    return (HA[:, None, :] != HB[None, :, :]).sum(axis=-1).astype(np.int64)


def hamming_hausdorff(HA, HB) -> int:
    """Haus^H(A, B): max of the two directed max-min Hamming distances."""
    return int(hausdorff_from_matrix(hamming_matrix(HA, HB)))


def full_scores(index, HQ) -> np.ndarray:
    """Haus^H of the query codes HQ to the codes of every set of the index."""
    H = index.H
    off = index.offsets
    return np.array([hamming_hausdorff(HQ, H[off[j]:off[j + 1]]) for j in range(index.n_sets)],
                    dtype=np.int64)


def full_candidates(scores: np.ndarray, c: int):
    """The first min(c, n) sets by (Haus^H, id): (ids, scores)."""
    scores = np.asarray(scores, dtype=np.int64)
    order = np.lexsort((np.arange(len(scores)), scores))[:c]
    return order.astype(np.int64), scores[order]


def search_full(index, Q, c: int, k: int) -> dict:
    """Alg. 2 for one query set Q [m_q, d]."""
    Q = np.asarray(Q, dtype=np.float64)
    HQ = codes(Q, index.idx, index.wta_k)
    scores = full_scores(index, HQ)
    f_ids, f_scores = full_candidates(scores, c)
    h2 = np.array([hausdorff_sq(Q, index.members(j)) for j in f_ids], dtype=np.float64)
    order = np.lexsort((f_ids, h2))[:k]
    ids, top_h2 = f_ids[order], h2[order]
    return dict(HQ=HQ, scores=scores, f_ids=f_ids, f_scores=f_scores, f_h2=h2,
                ids=ids, h2=top_h2, dist=np.sqrt(top_h2).astype(np.float32))
