"""Cascade search end to end (Alg. 6) and exact brute force (Def. 5).

build_index   codes for every database vector (Alg. 1), then the count and
              binary Bloom filter of every set (Algs. 3 and 5)
search        one query: query sketches, top-A positions, first filter,
              Hamming scores, the first T by (score, id), exact Hausdorff
              on those T, and the first k by (distance, id)
bruteforce    exact Hausdorff against every set, first k by (distance, id)
search_metric, bruteforce_metric
              the same with F2 (or every set) measured by MeanMin or Min
              distance (Sec. 3.2) instead of the Hausdorff distance

Ranking uses the squared Hausdorff distance in float64, which is exact for
inputs on the 2^-12 grid; reported distances are float32(sqrt(H^2)).  The
final step of Alg. 6 keeps every set whose distance is at most the k-th
smallest, which can return more than k sets on ties; here exactly
min(k, |F2|) sets are returned, ties to the lower id.  The loop of the
last steps runs over F2 (the survivors of the second layer).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import filter as flt
from .flyhash import codes
from .hausdorff import hausdorff_from_matrix, hausdorff_sq, mean_min_from_matrix, min_from_matrix, pairwise_sq
from .sketch import binary_bloom, count_bloom


@dataclass
class Index:
    X: np.ndarray          # float64 [N, d]
    offsets: np.ndarray    # int64 [n + 1]
    idx: np.ndarray        # [L, s] projection rows
    wta_k: int
    H: np.ndarray          # bool [N, L] per-vector codes
    C: np.ndarray          # int64 [n, L] count Bloom filters
    B: np.ndarray          # bool [n, L] binary Bloom filters (= sketches)

    @property
    def n_sets(self) -> int:
        return len(self.offsets) - 1

    def members(self, j: int) -> np.ndarray:
        return self.X[self.offsets[j]:self.offsets[j + 1]]


def build_index(X, offsets, idx, wta_k: int) -> Index:
    X = np.asarray(X, dtype=np.float64)
    offsets = np.asarray(offsets, dtype=np.int64)
    H = codes(X, idx, wta_k)
    return Index(X, offsets, np.asarray(idx), wta_k, H,
                 count_bloom(H, offsets), binary_bloom(H, offsets))


def rank_by_distance(ids: np.ndarray, h2: np.ndarray, k: int):
    order = np.lexsort((ids, h2))[:k]
    return ids[order], h2[order]


def search(index: Index, Q, A: int, M: int, T: int, k: int) -> dict:
    """One query set Q [m_q, d]; returns every intermediate of Alg. 6."""
    Q = np.asarray(Q, dtype=np.float64)
    return search_codes(index, Q, codes(Q, index.idx, index.wta_k), A, M, T, k)


def index_from_codes(X, offsets, H, wta_k: int) -> Index:
    """An index whose codes come from elsewhere (the learned projection)."""
    X = np.asarray(X, dtype=np.float64)
    offsets = np.asarray(offsets, dtype=np.int64)
    H = np.asarray(H, dtype=bool)
    return Index(X, offsets, np.zeros((0, 0), np.int64), wta_k, H, count_bloom(H, offsets), binary_bloom(H, offsets))


def search_codes(index: Index, Q, HQ, A: int, M: int, T: int, k: int) -> dict:
    """Alg. 6 for query Q with query codes HQ given."""
    Q = np.asarray(Q, dtype=np.float64)
    C_Q, S_Q = flt.query_sketches(HQ)
    P = flt.top_positions(C_Q, A)
    member = flt.first_filter(index.C, P, M)
    scores = flt.hamming(S_Q, index.B)
    f2_ids, f2_scores = flt.second_filter(member, scores, T)
    h2 = np.array([hausdorff_sq(Q, index.members(j)) for j in f2_ids], dtype=np.float64)
    ids, top_h2 = rank_by_distance(f2_ids, h2, k)
    return dict(HQ=HQ, C_Q=C_Q, S_Q=S_Q, P=P, member=member, scores=scores,
                f2_ids=f2_ids, f2_scores=f2_scores, f2_h2=h2,
                ids=ids, h2=top_h2, dist=np.sqrt(top_h2).astype(np.float32))


def all_hausdorff_sq(X, offsets, Q) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    n = len(offsets) - 1
    return np.array([hausdorff_sq(Q, X[offsets[j]:offsets[j + 1]]) for j in range(n)],
                    dtype=np.float64)


def bruteforce(X, offsets, Q, k: int):
    """Exact top-k by Hausdorff distance over all sets (Def. 5 with delta=0)."""
    h2 = all_hausdorff_sq(X, offsets, Q)
    ids, top_h2 = rank_by_distance(np.arange(len(h2)), h2, k)
    return ids, top_h2, np.sqrt(top_h2).astype(np.float32)


def recall_at_k(found, truth) -> float:
    """|R_k ∩ G_k| / |G_k| (Sec. 6.1.3)."""
    truth = set(int(t) for t in truth)
    return len(truth & set(int(f) for f in found)) / max(1, len(truth))


# ---------------------------------------------------------------------------
# Other set measures in the re-rank (Sec. 3.2 defines Min and MeanMin beside
# the Hausdorff distance; Sec. 6 searches with MeanMin in place of it).  The
# filter layers are the same; only the measure of F2's sets changes.

METRICS = ("hausdorff", "meanmin", "min")


def set_key(Q, V, metric: str) -> float:
    """Ranking key of set V for query set Q.

    hausdorff: squared Hausdorff distance (Def. 4), exact on the grid
    min:       smallest squared distance between the sets, exact on the grid
    meanmin:   MeanMin from Q to V, the mean over q in Q of min over v of
               |q - v| (not squared), rounded to float32: the measure is a
               mean of square roots, so the ranking decision is taken on the
               float32 value (ties to the lower id), the precision of the
               reported distance."""
    D2 = pairwise_sq(Q, V)
    if metric == "hausdorff":
        return hausdorff_from_matrix(D2)
    if metric == "min":
        return min_from_matrix(D2)
    if metric == "meanmin":
        return float(np.float32(mean_min_from_matrix(np.sqrt(D2))))
    raise ValueError(metric)


def key_to_distance(key: np.ndarray, metric: str) -> np.ndarray:
    key = np.asarray(key, dtype=np.float64)
    return (key if metric == "meanmin" else np.sqrt(key)).astype(np.float32)


def search_metric(index: Index, Q, A: int, M: int, T: int, k: int, metric: str) -> dict:
    """Alg. 6 with the last steps measuring F2's sets by `metric`."""
    Q = np.asarray(Q, dtype=np.float64)
    r = search_codes(index, Q, codes(Q, index.idx, index.wta_k), A, M, T, k)
    keys = np.array([set_key(Q, index.members(j), metric) for j in r["f2_ids"]], dtype=np.float64)
    ids, top = rank_by_distance(r["f2_ids"], keys, k)
    r.update(f2_keys=keys, ids=ids, keys=top, dist=key_to_distance(top, metric))
    return r


def bruteforce_metric(X, offsets, Q, k: int, metric: str):
    """Exact top-k over all sets by `metric`: (ids, keys, float32 distances)."""
    X = np.asarray(X, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    n = len(offsets) - 1
    keys = np.array([set_key(Q, X[offsets[j]:offsets[j + 1]], metric) for j in range(n)], dtype=np.float64)
    ids, top = rank_by_distance(np.arange(n), keys, k)
    return ids, top, key_to_distance(top, metric)
