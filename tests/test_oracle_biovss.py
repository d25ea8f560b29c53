"""Pins of the oracle's full-scan search (Alg. 2): the Hamming form of the
Hausdorff distance over codes, the first-c candidate set, and the whole
search."""
import itertools

import numpy as np
import pytest
from scipy.spatial.distance import hamming as scipy_hamming

from oracle import biovss, prng, search
from paper_2412_03301_amd import synth


def _codes(strings):
    return np.array([[ch == "1" for ch in s] for s in strings], dtype=bool)


def test_hand_computed_example():
    # positions 0..7 left to right; every code has two ones.
    Q = _codes(["11000000", "00110000"])
    V = _codes(["10100000", "00001100", "01010000"])
    # q1 = {0,1}: v1 = {0,2} differs at 1, 2 -> 2; v2 = {4,5} -> 4; v3 = {1,3} -> 2
    # q2 = {2,3}: v1 -> 2; v2 -> 4; v3 -> 2
    assert biovss.hamming_matrix(Q, V).tolist() == [[2, 4, 2], [2, 4, 2]]
    # rows (query to set): minima 2, 2 -> 2; columns (set to query): v2's
    # nearest query code is 4 away -> 4; Haus^H = max(2, 4)
    assert biovss.hamming_hausdorff(Q, V) == 4
    assert biovss.hamming_hausdorff(V, Q) == 4
    # the one-directional term alone would give 2: the example tells them apart
    assert biovss.hamming_matrix(Q, V).min(axis=1).max() == 2


def _random_code_sets(rng, count, m_lo, m_hi, L, k):
    out = []
    for _ in range(count):
        m = int(rng.integers(m_lo, m_hi + 1))
        H = np.zeros((m, L), dtype=bool)
        for i in range(m):
            H[i, rng.choice(L, size=k, replace=False)] = True
        out.append(H)
    return out


def test_singletons_reduce_to_plain_hamming():
    rng = np.random.default_rng(1)
    sets = _random_code_sets(rng, 8, 1, 1, 128, 9)
    for a, b in itertools.combinations(sets, 2):
        assert biovss.hamming_hausdorff(a, b) == round(scipy_hamming(a[0], b[0]) * 128)


def test_overlap_closed_form_with_python_integers():
    # With exactly k ones per code: Hamming = 2 k - 2 |a AND b|, counted here
    # on Python integers independently of the boolean matrices.
    rng = np.random.default_rng(2)
    L, k = 256, 17
    A, B = _random_code_sets(rng, 2, 5, 9, L, k)
    ia = [int("".join("1" if x else "0" for x in row), 2) for row in A]
    ib = [int("".join("1" if x else "0" for x in row), 2) for row in B]
    want = [[2 * k - 2 * bin(x & y).count("1") for y in ib] for x in ia]
    assert biovss.hamming_matrix(A, B).tolist() == want


def test_metric_invariants():
    rng = np.random.default_rng(3)
    sets = _random_code_sets(rng, 8, 1, 6, 64, 7)
    for A in sets:
        assert biovss.hamming_hausdorff(A, A) == 0
    for A, B in itertools.combinations(sets, 2):
        assert biovss.hamming_hausdorff(A, B) == biovss.hamming_hausdorff(B, A)
    for A, B, C in itertools.permutations(sets[:5], 3):
        assert biovss.hamming_hausdorff(A, C) <= biovss.hamming_hausdorff(A, B) + biovss.hamming_hausdorff(B, C)


def test_candidates_first_c_by_score_then_id():
    scores = np.array([5, 3, 3, 9, 0, 3, 5])
    ids, sc = biovss.full_candidates(scores, 4)
    assert ids.tolist() == [4, 1, 2, 5] and sc.tolist() == [0, 3, 3, 3]
    ids, _ = biovss.full_candidates(scores, 100)
    assert ids.tolist() == sorted(range(7), key=lambda j: (scores[j], j))


@pytest.fixture(scope="module")
def small_index():
    db = synth.make_database(120, 2, 9, 32, n_topics=6, seed=4)
    X = db.vectors.numpy().astype(np.float64)
    ix = search.build_index(X, db.offsets, prng.projection_rows(4, 32, 256, 4), 12)
    q, q_off, _ = synth.make_subset_queries(db, 3, seed=5)
    return ix, q.numpy().astype(np.float64), q_off


def test_full_scan_with_every_set_is_brute_force(small_index):
    ix, q, q_off = small_index
    for i in range(3):
        Q = q[q_off[i]:q_off[i + 1]]
        r = biovss.search_full(ix, Q, c=ix.n_sets, k=10)
        ids, h2, _ = search.bruteforce(ix.X, ix.offsets, Q, 10)
        assert r["ids"].tolist() == ids.tolist()
        assert np.array_equal(r["h2"], h2)


def test_full_scan_scores_match_codes_of_members(small_index):
    ix, q, q_off = small_index
    Q = q[q_off[0]:q_off[1]]
    r = biovss.search_full(ix, Q, c=15, k=5)
    assert len(r["f_ids"]) == 15 and len(r["ids"]) == 5
    for j in (0, 7, 50, 119):
        V = ix.H[ix.offsets[j]:ix.offsets[j + 1]]
        D = [[int((a != b).sum()) for b in V] for a in r["HQ"]]
        want = max(max(min(row) for row in D), max(min(col) for col in zip(*D)))
        assert r["scores"][j] == want
    # a set whose member codes include every query code is at Haus^H = its
    # farthest member's distance to the query codes, never below 0
    assert (r["scores"] >= 0).all() and (r["scores"] <= 2 * ix.wta_k).all()
    # the results come from the candidates, in (distance, id) order
    assert set(r["ids"].tolist()) <= set(r["f_ids"].tolist())
    assert all((a, b) <= (c, d) for (a, b), (c, d) in zip(zip(r["h2"], r["ids"]), zip(r["h2"][1:], r["ids"][1:])))
