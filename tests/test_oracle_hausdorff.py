"""Pins of the oracle's set distances (Def. 4, Sec. 3.2, Lemma 1)."""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist, directed_hausdorff

from oracle import hausdorff as hd
from tests.conftest import GOLDEN

EX = json.load(open(os.path.join(GOLDEN, "distance_examples.json")))


def test_precision_example_printed_values():
    pa = EX["precision"]
    QA = np.array(pa["Q_to_A"], float)   # rows A_i, columns Q_j
    QB = np.array(pa["Q_to_B"], float)
    pr = pa["printed"]
    assert hd.min_from_matrix(QA) == pr["d_min(Q,A)"]
    assert hd.min_from_matrix(QB) == pr["d_min(Q,B)"]
    # MeanMin from Q: average over Q items (the columns) of their minimum.
    assert hd.mean_min_from_matrix(QA.T) == pr["d_mean_min(Q,A)"]
    assert hd.mean_min_from_matrix(QB.T) == pr["d_mean_min(Q,B)"]
    assert hd.hausdorff_from_matrix(QA) == pr["d_H(Q,A)"]
    # The printed 2 disagrees with Def. 4 on the printed matrix; the
    # definition gives 1.
    assert hd.hausdorff_from_matrix(QB) == pa["by_definition"]["d_H(Q,B)"]
    assert hd.hausdorff_from_matrix(QB) != pr["d_H(Q,B)"]


def test_symmetry_example_printed_values():
    sy = EX["symmetry"]
    QA = np.array(sy["Q_to_A"], float)
    pr = sy["printed"]
    assert hd.min_from_matrix(QA) == pr["d_min(Q,A)"] == hd.min_from_matrix(QA.T)
    assert hd.mean_min_from_matrix(QA.T) == pr["d_mean_min(Q,A)"]
    assert round(hd.mean_min_from_matrix(QA), 2) == pr["d_mean_min(A,Q)"]
    assert hd.hausdorff_from_matrix(QA) == pr["d_H(Q,A)"]
    assert hd.hausdorff_from_matrix(QA.T) == pr["d_H(A,Q)"]


def test_example2_aggregation():
    ex = EX["example2"]
    # Q has 3 items (rows), V has 2 (columns); directed terms 3 and 2.
    D = np.array([[2.0, 4.0], [3.0, 5.0], [4.0, 2.0]])
    assert hd.directed_from_matrix(D) == ex["directed_Q_to_V"]
    assert hd.directed_from_matrix(D.T) == ex["directed_V_to_Q"]
    assert hd.hausdorff_from_matrix(D) == ex["hausdorff"]


def _grid_sets(rng, count, m_lo, m_hi, d):
    out = []
    for _ in range(count):
        m = int(rng.integers(m_lo, m_hi + 1))
        x = rng.standard_normal((m, d))
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out.append(np.round(x * 4096) / 4096)
    return out


def test_agrees_with_scipy_directed_hausdorff():
    rng = np.random.default_rng(1)
    sets = _grid_sets(rng, 12, 1, 9, 16)
    for Q, V in itertools.product(sets[:6], sets[6:]):
        ref = max(directed_hausdorff(Q, V)[0], directed_hausdorff(V, Q)[0])
        assert math.isclose(hd.hausdorff(Q, V), ref, rel_tol=1e-12, abs_tol=1e-12)


def test_metric_invariants():
    rng = np.random.default_rng(2)
    sets = _grid_sets(rng, 9, 1, 7, 8)
    for A in sets:
        assert hd.hausdorff_sq(A, A) == 0.0
    for A, B in itertools.combinations(sets, 2):
        assert hd.hausdorff_sq(A, B) == hd.hausdorff_sq(B, A)
    for A, B, C in itertools.permutations(sets[:6], 3):
        assert hd.hausdorff(A, C) <= hd.hausdorff(A, B) + hd.hausdorff(B, C) + 1e-12


def test_singletons_reduce_to_euclidean():
    rng = np.random.default_rng(3)
    a, b = _grid_sets(rng, 2, 1, 1, 32)
    assert math.isclose(hd.hausdorff(a, b), float(np.linalg.norm(a[0] - b[0])), rel_tol=1e-14)


def test_lemma1_bounds_distance_form():
    # Lemma 1 bounds a min-max aggregate by the extreme entries; in
    # distance form: min_ij d_ij <= H <= max_ij d_ij.
    rng = np.random.default_rng(4)
    sets = _grid_sets(rng, 8, 2, 6, 8)
    for A, B in itertools.combinations(sets, 2):
        D = cdist(A, B)
        h = hd.hausdorff(A, B)
        assert D.min() - 1e-12 <= h <= D.max() + 1e-12


def test_exact_on_grid_against_integer_brute_force():
    # 4096 x is an integer on the grid, so 2^24 H^2 is an integer that pure
    # Python integers compute with no rounding at all.
    rng = np.random.default_rng(5)
    sets = _grid_sets(rng, 6, 1, 5, 12)
    for A, B in itertools.combinations(sets, 2):
        ia = [[int(round(v * 4096)) for v in row] for row in A]
        ib = [[int(round(v * 4096)) for v in row] for row in B]
        d2 = [[sum((x - y) ** 2 for x, y in zip(p, q)) for q in ib] for p in ia]
        h2_int = max(max(min(r) for r in d2), max(min(d2[i][j] for i in range(len(ia)))
                                                   for j in range(len(ib))))
        assert hd.hausdorff_sq(A, B) * 2 ** 24 == h2_int


@pytest.mark.parametrize("mistake", ["one_direction", "min_of_mins", "max_of_max"])
def test_pins_catch_plausible_mistakes(mistake):
    # The printed examples tell apart the usual slips in Def. 4.
    D = np.array(EX["symmetry"]["Q_to_A"], float)
    wrong = {
        "one_direction": D.T.min(axis=1).max(),
        "min_of_mins": D.min(),
        "max_of_max": D.max(),
    }[mistake]
    assert wrong != EX["symmetry"]["printed"]["d_H(Q,A)"]
