"""Set distances (Def. 4 and the comparison measures of Sec. 3.2).

A distance matrix D here always has the items of the first set on its
rows and the items of the second set on its columns: D[i, j] = d(a_i, b_j).

Hausdorff (Def. 4):  max( max_i min_j D[i, j],  max_j min_i D[i, j] )
Min distance:        min_{i, j} D[i, j]
MeanMin (A to B):    (1 / |A|) * sum_i min_j D[i, j]

For point sets the oracle works on squared Euclidean distances in float64
and takes one square root at the end; the square root is monotone, so the
max/min structure of Def. 4 is the same on squared values.  For inputs on
the 2^-12 grid with norms of at most 2 every squared distance is an
integer multiple of 2^-24 below 16, so these float64 values are exact.
"""
from __future__ import annotations

import numpy as np


def pairwise_sq(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances [|A|, |B|], summed from differences."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    diff = A[:, None, :] - B[None, :, :]
    return (diff * diff).sum(axis=-1)


def hausdorff_from_matrix(D: np.ndarray) -> float:
    D = np.asarray(D, dtype=np.float64)
    return float(max(D.min(axis=1).max(), D.min(axis=0).max()))


def directed_from_matrix(D: np.ndarray) -> float:
    """max over rows of the row minimum: the row set's directed distance."""
    return float(np.asarray(D, dtype=np.float64).min(axis=1).max())


def min_from_matrix(D: np.ndarray) -> float:
    return float(np.asarray(D, dtype=np.float64).min())


def mean_min_from_matrix(D: np.ndarray) -> float:
    return float(np.asarray(D, dtype=np.float64).min(axis=1).mean())


def hausdorff_sq(Q: np.ndarray, V: np.ndarray) -> float:
    """Squared Hausdorff distance between two point sets."""
    return hausdorff_from_matrix(pairwise_sq(Q, V))


def hausdorff(Q: np.ndarray, V: np.ndarray) -> float:
    return float(np.sqrt(hausdorff_sq(Q, V)))
