"""Pins of the oracle's projection and winner-take-all codes (Def. 7, Alg. 1)."""
import json
import os

import numpy as np
import pytest

from oracle import flyhash, prng
from tests.conftest import GOLDEN

SM = json.load(open(os.path.join(GOLDEN, "splitmix64_vectors.json")))


def test_splitmix64_known_answers():
    r = prng.SplitMix64(1234567)
    assert [r.next() for _ in range(5)] == SM["seed_1234567"]
    assert prng.SplitMix64(0).next() == int(SM["seed_0_first"], 16)


@pytest.mark.parametrize("d,L,s", [(128, 1024, 8), (384, 4096, 16), (5, 64, 5), (17, 128, 1)])
def test_projection_rows_invariants(d, L, s):
    idx = prng.projection_rows(7, d, L, s)
    assert idx.shape == (L, s)
    assert idx.min() >= 0 and idx.max() < d
    for row in idx:
        assert len(set(row.tolist())) == s
        assert (np.diff(row) > 0).all() if s > 1 else True
    if s == d:
        assert (idx == np.arange(d)[None, :]).all()


def test_projection_dimension_histogram_is_uniform():
    d, L, s = 384, 4096, 16
    idx = prng.projection_rows(0, d, L, s)
    counts = np.bincount(idx.ravel(), minlength=d)
    expected = L * s / d
    chi2 = ((counts - expected) ** 2 / expected).sum()
    # 383 degrees of freedom: mean 383, sd ~27.7; 6 sd is a loose bound.
    assert chi2 < 383 + 6 * 27.7


def test_projection_depends_on_seed():
    a = prng.projection_rows(0, 64, 256, 4)
    b = prng.projection_rows(1, 64, 256, 4)
    assert (a != b).any()


def test_hand_computed_code():
    # d = 4, L = 4, s = 2: y = (x0+x1, x1+x2, x2+x3, x0+x3).
    idx = np.array([[0, 1], [1, 2], [2, 3], [0, 3]])
    x = np.array([[0.5, 0.25, -0.25, 0.75]])
    y = flyhash.project(x, idx)
    assert y.tolist() == [[0.75, 0.0, 0.5, 1.25]]
    assert flyhash.wta(y, 2).tolist() == [[True, False, False, True]]
    assert flyhash.wta(y, 1).tolist() == [[False, False, False, True]]
    assert flyhash.wta(y, 3).tolist() == [[True, False, True, True]]


def test_ties_go_to_lower_index():
    idx = np.array([[0, 1], [1, 2], [2, 3], [0, 3]])
    x = np.full((1, 4), 0.5)
    y = flyhash.project(x, idx)
    assert (y == 1.0).all()
    assert flyhash.wta(y, 2).tolist() == [[True, True, False, False]]


def _grid(rng, n, d):
    x = rng.standard_normal((n, d))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return np.round(x * 4096) / 4096


def test_wta_matches_full_sort_brute_force():
    rng = np.random.default_rng(0)
    d, L, s, k = 16, 64, 3, 7
    idx = prng.projection_rows(3, d, L, s)
    X = _grid(rng, 40, d)
    # Force many ties: quantise a copy coarsely.
    X[20:] = np.round(X[20:] * 4) / 4
    H = flyhash.codes(X, idx, k)
    for x, h in zip(X, H):
        y = [sum(float(x[i]) for i in idx[j]) for j in range(L)]
        winners = sorted(range(L), key=lambda j: (-y[j], j))[:k]
        assert sorted(np.flatnonzero(h).tolist()) == sorted(winners)


def test_exactly_k_bits_and_extremes():
    rng = np.random.default_rng(1)
    d, L, s = 32, 256, 4
    idx = prng.projection_rows(5, d, L, s)
    X = _grid(rng, 50, d)
    for k in (1, 17, 64, L):
        H = flyhash.codes(X, idx, k)
        assert (H.sum(axis=1) == k).all()
    assert flyhash.codes(X, idx, L).all()


def test_all_inputs_summed_gives_lowest_indices():
    # s = d: every output is the same sum, so the code is the first k outputs.
    rng = np.random.default_rng(2)
    d, L, k = 8, 128, 10
    idx = prng.projection_rows(1, d, L, d)
    H = flyhash.codes(_grid(rng, 5, d), idx, k)
    assert (H[:, :k]).all() and not H[:, k:].any()


def test_code_is_scale_invariant_on_grid():
    rng = np.random.default_rng(3)
    d, L, s, k = 64, 512, 8, 16
    idx = prng.projection_rows(2, d, L, s)
    X = _grid(rng, 30, d)
    assert (flyhash.codes(X, idx, k) == flyhash.codes(2 * X, idx, k)).all()


def test_pack_bit_order():
    H = np.zeros((3, 128), bool)
    H[0, 0] = H[1, 63] = H[2, 64] = True
    W = flyhash.pack(H)
    assert W.dtype == np.uint64 and W.shape == (3, 2)
    assert W[0].tolist() == [1, 0]
    assert W[1].tolist() == [1 << 63, 0]
    assert W[2].tolist() == [0, 1]
    assert (flyhash.unpack(W, 128) == H).all()
