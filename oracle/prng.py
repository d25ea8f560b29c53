"""Random sparse binary projection (oracle side).

Def. 7 of the paper only says that W in R^{b x d} is a random projection
matrix.  The construction used throughout this project: every row of W
holds exactly ``fan_in`` ones at distinct input dimensions drawn
uniformly without replacement, rows independent.  The draws come from one
splitmix64 stream (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) seeded with ``seed``; a bounded integer
in [0, d) is the high 32 bits of a draw times d, shifted right by 32
(Lemire's multiply-shift reduction); a dimension already in the row is
rejected and redrawn; rows are consumed in order 0..L-1 and each row is
stored sorted ascending.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    """splitmix64: Weyl increment, then two xor-shift-multiply rounds."""

    def __init__(self, seed: int):
        self.state = int(seed) & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)


def projection_rows(seed: int, dim: int, code_bits: int, fan_in: int) -> np.ndarray:
    """idx[L][s]: the input dimensions summed by each of the L outputs."""
    if not (1 <= fan_in <= dim):
        raise ValueError("fan_in must lie in [1, dim]")
    rng = SplitMix64(seed)
    idx = np.empty((code_bits, fan_in), dtype=np.int64)
    for j in range(code_bits):
        row: list[int] = []
        while len(row) < fan_in:
            i = ((rng.next() >> 32) * dim) >> 32
            if i not in row:
                row.append(i)
        idx[j] = sorted(row)
    return idx


def projection_matrix(idx: np.ndarray, dim: int) -> np.ndarray:
    """Dense 0/1 matrix W (float64, L x d) with W[j, idx[j, :]] = 1."""
    L, s = idx.shape
    W = np.zeros((L, dim), dtype=np.float64)
    W[np.repeat(np.arange(L), s), idx.reshape(-1)] = 1.0
    return W
