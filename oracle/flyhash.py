"""FlyHash codes: h = WTA(W v) (Def. 7; Alg. 1, Gen_Binary_Codes).

The winner-take-all step keeps the L_wta largest projected values as 1.
The paper does not say how equal values are ordered; here a tie goes to
the lower output index, so every code has exactly L_wta ones.
"""
from __future__ import annotations

import numpy as np

from .prng import projection_matrix


def project(X: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """W x for each row x of X, in float64 (Alg. 1, matrix projection)."""
    X = np.asarray(X, dtype=np.float64)
    W = projection_matrix(idx, X.shape[1])
    return X @ W.T


def wta(Y: np.ndarray, wta_k: int) -> np.ndarray:
    """Winner-take-all: boolean [N, L] with the wta_k largest of each row.

    A stable sort of -y keeps equal values in ascending index order, so
    the lowest indices win ties."""
    order = np.argsort(-Y, axis=1, kind="stable")[:, :wta_k]
    H = np.zeros(Y.shape, dtype=bool)
    np.put_along_axis(H, order, True, axis=1)
    return H


def codes(X: np.ndarray, idx: np.ndarray, wta_k: int) -> np.ndarray:
    """Sparse binary codes of the rows of X (Alg. 1), boolean [N, L]."""
    return wta(project(X, idx), wta_k)


def pack(H: np.ndarray) -> np.ndarray:
    """Pack boolean codes [N, L] into uint64 words [N, L/64]; output j is
    bit (j % 64) of word j // 64."""
    H = np.asarray(H, dtype=bool)
    by = np.packbits(H, axis=-1, bitorder="little")
    return np.ascontiguousarray(by).view("<u8")


def unpack(words: np.ndarray, code_bits: int) -> np.ndarray:
    by = np.ascontiguousarray(words).view(np.uint8)
    return np.unpackbits(by, axis=-1, bitorder="little", count=code_bits).astype(bool)
