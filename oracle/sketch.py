"""Per-set Bloom sketches (Defs. 8 and 10; Algs. 3 and 5).

count Bloom filter  C^(j) = sum of the member codes (Def. 8, Alg. 3)
binary Bloom filter B^(j) = OR of the member codes (Def. 10, Alg. 5);
the set sketch S^(j) is B^(j) itself.
"""
from __future__ import annotations

import numpy as np


def count_bloom(H: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """int64 [n, L]: per set, how many member codes have each bit set."""
    n = len(offsets) - 1
    C = np.zeros((n, H.shape[1]), dtype=np.int64)
    for j in range(n):
        C[j] = H[offsets[j]:offsets[j + 1]].sum(axis=0)
    return C


def binary_bloom(H: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """bool [n, L]: per set, the bitwise OR of the member codes."""
    n = len(offsets) - 1
    B = np.zeros((n, H.shape[1]), dtype=bool)
    for j in range(n):
        B[j] = H[offsets[j]:offsets[j + 1]].any(axis=0)
    return B
