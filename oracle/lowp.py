"""Low-precision re-rank of the cascade search (test infrastructure).

The paper computes Hausdorff distances (Def. 4) in full precision.  The
precision form quantises database and query vectors, computes the pairwise
dot products of the quantised values, and re-checks exactly every
candidate whose approximate distance lies within a relative margin of the
k-th approximate distance; the final top-k comes from the exact values.

Encodings, written from their published definitions:
  bfloat16   the upper 16 bits of an IEEE float32, rounded to nearest,
             ties to even
  e4m3       OCP 8-bit float E4M3 ("FN"): 1 sign, 4 exponent (bias 7) and
             3 mantissa bits; normal values 2^(e-7) * (1 + m/8) for
             e = 1..15 (e = 15, m = 7 is NaN, so the largest value is 448),
             subnormals m * 2^-9; no infinities.  Rounded to nearest, ties
             to even.
FP8 vectors carry a scale per set: s = float32(max |x| over the set) /
float32(448), and each component is stored as e4m3(clamp(x / s, +-448)),
all in float32 arithmetic.  BF16 needs no scale.

Approximate squared distance of rows x (set scale s_x) and y (s_y):
    D~2 = |x|^2 + |y|^2 - 2 s_x s_y (x~ . y~),   clamped at 0,
with exact norms of the unquantised rows and the dot product of the
decoded quantised values, in float64 here (float32 accumulation on the
GPU).  The approximate Hausdorff value takes Def. 4's max/min structure
over D~2.
"""
from __future__ import annotations

import numpy as np

from . import filter as flt
from .flyhash import codes
from .hausdorff import hausdorff_sq

E4M3_MAX = 448.0


def bf16_bits(x) -> np.ndarray:
    """bfloat16 bit patterns of float32 values (round to nearest even)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return (u >> 16).astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def e4m3_bits(x) -> np.ndarray:
    """E4M3 bit patterns of float32 values with |x| <= 448 (round to
    nearest even).  Larger magnitudes are rejected: callers clamp first."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    if np.any(np.abs(x) > E4M3_MAX) or np.any(~np.isfinite(x)):
        raise ValueError("e4m3 input outside +-448")
    sign = (x < 0).astype(np.uint8) << 7
    a = np.abs(x)
    out = np.zeros(a.shape, dtype=np.uint8)
    sub = a < 2.0 ** -6
    # subnormal range: multiples of 2^-9; a code of 8 is the smallest normal
    out[sub] = np.rint(a[sub] * 512.0).astype(np.uint8)
    nrm = ~sub
    if np.any(nrm):
        an = a[nrm]
        e = np.floor(np.log2(an)).astype(np.int64)
        # guard log2 rounding at exact powers of two
        e = np.where(2.0 ** e > an, e - 1, e)
        e = np.where(2.0 ** (e + 1) <= an, e + 1, e)
        m = np.rint((an / 2.0 ** e - 1.0) * 8.0).astype(np.int64)
        carry = m == 8
        e = np.where(carry, e + 1, e)
        m = np.where(carry, 0, m)
        out[nrm] = (((e + 7) << 3) | m).astype(np.uint8)
    return out | sign


def e4m3_value(bits) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint8).astype(np.int64)
    s = np.where(b & 0x80, -1.0, 1.0)
    e = (b >> 3) & 0xF
    m = b & 7
    if np.any((e == 15) & (m == 7)):
        raise ValueError("e4m3 NaN")
    v = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * 2.0 ** (e - 7))
    return s * v


def fp8_scale(rows) -> np.float32:
    """Scale of one set: float32(max |x|) / float32(448); 1 for an all-zero set."""
    mx = np.float32(np.max(np.abs(np.asarray(rows, dtype=np.float32)))) if np.size(rows) else np.float32(0)
    return np.float32(1.0) if mx == 0 else np.float32(mx / np.float32(E4M3_MAX))


def quantise(rows, fmt: str):
    """(decoded quantised rows float64, scale) of one set."""
    r = np.asarray(rows, dtype=np.float32)
    if fmt == "bf16":
        return bf16_value(bf16_bits(r)), 1.0
    if fmt == "fp8":
        s = fp8_scale(r)
        t = np.clip(r / s, np.float32(-E4M3_MAX), np.float32(E4M3_MAX))
        return e4m3_value(e4m3_bits(t)), float(s)
    raise ValueError(fmt)


def approx_pairwise_sq(Q, V, fmt: str) -> np.ndarray:
    """D~2 [|Q|, |V|] of two sets (each quantised with its own scale)."""
    Q = np.asarray(Q, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    qq, sq = quantise(Q, fmt)
    vv, sv = quantise(V, fmt)
    nq = (Q * Q).sum(axis=1)
    nv = (V * V).sum(axis=1)
    D = nq[:, None] + nv[None, :] - 2.0 * sq * sv * (qq @ vv.T)
    return np.maximum(D, 0.0)


def approx_hausdorff_sq(Q, V, fmt: str) -> float:
    D = approx_pairwise_sq(Q, V, fmt)
    return float(max(D.min(axis=1).max(), D.min(axis=0).max()))


def recheck_threshold(h2_kth: float, margin: float) -> np.float32:
    """Squared-distance threshold of the re-check, every step in float32:
    distances within (1 + margin) of the k-th approximate distance.

    A distance d is within the margin when d <= (1 + margin) d_k, that is
    d^2 <= (1 + margin)^2 d_k^2 (both sides are non-negative), so the test
    runs on squared values against the k-th squared value times the square
    of the factor.  The steps are float32, as on the GPU, so that a value
    right at the threshold is decided the same way on both sides."""
    f1 = np.float32(1.0) + np.float32(margin)
    return np.float32(np.float32(h2_kth) * np.float32(f1 * f1))


def select_recheck(ids, ah2, k: int, margin: float) -> np.ndarray:
    """Candidates to re-check exactly: in (approximate value, id) order,
    those whose approximate squared value (as float32) is at most the
    threshold of the k-th one; all of them when there are fewer than k."""
    ids = np.asarray(ids)
    ah2 = np.asarray(ah2, dtype=np.float64)
    order = np.lexsort((ids, ah2))
    if len(ids) < k:
        return ids[order]
    thr = recheck_threshold(ah2[order[k - 1]], margin)
    return ids[order][ah2[order].astype(np.float32) <= thr]


def search_lowp(index, Q, A: int, M: int, T: int, k: int, fmt: str, margin: float) -> dict:
    """Alg. 6 with the precision form of the re-rank."""
    Q = np.asarray(Q, dtype=np.float64)
    HQ = codes(Q, index.idx, index.wta_k)
    C_Q, S_Q = flt.query_sketches(HQ)
    P = flt.top_positions(C_Q, A)
    member = flt.first_filter(index.C, P, M)
    scores = flt.hamming(S_Q, index.B)
    f2_ids, _ = flt.second_filter(member, scores, T)
    ah2 = np.array([approx_hausdorff_sq(Q, index.members(j), fmt) for j in f2_ids], dtype=np.float64)
    recheck = select_recheck(f2_ids, ah2, k, margin)
    h2 = np.array([hausdorff_sq(Q, index.members(j)) for j in recheck], dtype=np.float64)
    o2 = np.lexsort((recheck, h2))[:k]
    return dict(f2_ids=f2_ids, approx_h2=ah2, recheck=recheck, ids=recheck[o2], h2=h2[o2],
                dist=np.sqrt(h2[o2]).astype(np.float32))
