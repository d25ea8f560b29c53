"""Pins of the oracle's point-set measures for the re-rank (Sec. 3.2: Min,
MeanMin and Hausdorff distances) and of their top-k ranking."""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.distance import cdist

from oracle import search
from tests.conftest import GOLDEN

EX = json.load(open(os.path.join(GOLDEN, "distance_examples.json")))


def _points_for_matrix(rows, D):
    """Plane points realising a printed distance matrix: Q1 = (0, 0),
    Q2 = (D, 0), and for every row (r1, r2) the point at distance r1 from Q1
    and r2 from Q2 (upper intersection of the two circles)."""
    Q = np.array([[0.0, 0.0], [D, 0.0]])
    pts = []
    for r1, r2 in rows:
        x = (r1 * r1 - r2 * r2 + D * D) / (2 * D)
        pts.append([x, math.sqrt(max(r1 * r1 - x * x, 0.0))])
    return Q, np.array(pts)


def test_printed_precision_example_from_points():
    pa = EX["precision"]
    pr = pa["printed"]
    # one shared Q (|Q1 Q2| = 5 fits every row of both matrices)
    Q, A = _points_for_matrix(pa["Q_to_A"], 5.0)
    _, B = _points_for_matrix(pa["Q_to_B"], 5.0)
    assert np.allclose(cdist(A, Q), np.array(pa["Q_to_A"], float), atol=1e-12)
    assert np.allclose(cdist(B, Q), np.array(pa["Q_to_B"], float), atol=1e-12)
    assert math.isclose(search.set_key(Q, A, "meanmin"), pr["d_mean_min(Q,A)"], rel_tol=1e-6)
    assert math.isclose(search.set_key(Q, B, "meanmin"), pr["d_mean_min(Q,B)"], rel_tol=1e-6)
    assert math.isclose(math.sqrt(search.set_key(Q, A, "min")), pr["d_min(Q,A)"], rel_tol=1e-12)
    assert math.isclose(math.sqrt(search.set_key(Q, B, "min")), pr["d_min(Q,B)"], rel_tol=1e-12)
    assert math.isclose(math.sqrt(search.set_key(Q, A, "hausdorff")), pr["d_H(Q,A)"], rel_tol=1e-12)
    assert math.isclose(math.sqrt(search.set_key(Q, B, "hausdorff")), pa["by_definition"]["d_H(Q,B)"],
                        rel_tol=1e-12)


def test_printed_symmetry_example_from_points():
    sy = EX["symmetry"]
    pr = sy["printed"]
    Q, A = _points_for_matrix(sy["Q_to_A"], 4.5)
    assert np.allclose(cdist(A, Q), np.array(sy["Q_to_A"], float), atol=1e-12)
    assert math.isclose(search.set_key(Q, A, "meanmin"), pr["d_mean_min(Q,A)"], rel_tol=1e-6)
    # the other direction: the mean over A's three points (printed rounded)
    assert round(search.set_key(A, Q, "meanmin"), 2) == pr["d_mean_min(A,Q)"]
    assert math.isclose(math.sqrt(search.set_key(Q, A, "min")), pr["d_min(Q,A)"], rel_tol=1e-12)
    assert search.set_key(Q, A, "min") == search.set_key(A, Q, "min")
    assert math.isclose(math.sqrt(search.set_key(Q, A, "hausdorff")), pr["d_H(Q,A)"], rel_tol=1e-12)


def _grid_sets(rng, count, m_lo, m_hi, d):
    out = []
    for _ in range(count):
        m = int(rng.integers(m_lo, m_hi + 1))
        x = rng.standard_normal((m, d))
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out.append(np.round(x * 4096) / 4096)
    return out


def test_singleton_query_is_nearest_neighbour_distance():
    # |Q| = 1: MeanMin and Min both reduce to the nearest-neighbour distance
    # of the one query vector, which a k-d tree finds independently.
    rng = np.random.default_rng(7)
    sets = _grid_sets(rng, 8, 1, 30, 16)
    for q, V in itertools.product([s[:1] for s in sets[:4]], sets[4:]):
        nn = cKDTree(V).query(q[0])[0]
        assert math.isclose(search.set_key(q, V, "meanmin"), float(np.float32(nn)), rel_tol=1e-7)
        assert math.isclose(math.sqrt(search.set_key(q, V, "min")), nn, rel_tol=1e-12)


def test_agrees_with_scipy_distance_matrix_and_order_relations():
    rng = np.random.default_rng(8)
    sets = _grid_sets(rng, 10, 1, 12, 24)
    for Q, V in itertools.product(sets[:5], sets[5:]):
        D = cdist(Q, V)
        mm = search.set_key(Q, V, "meanmin")
        mn = math.sqrt(search.set_key(Q, V, "min"))
        h = math.sqrt(search.set_key(Q, V, "hausdorff"))
        assert math.isclose(mm, float(np.float32(D.min(axis=1).mean())), rel_tol=1e-7)
        assert math.isclose(mn, D.min(), rel_tol=1e-12)
        # Min <= MeanMin <= directed Q->V term <= Hausdorff
        assert mn <= mm * (1 + 1e-7) and mm <= D.min(axis=1).max() * (1 + 1e-7) <= h * (1 + 1e-7)
    for A in sets:
        assert search.set_key(A, A, "meanmin") == 0.0 and search.set_key(A, A, "min") == 0.0


def test_meanmin_is_not_symmetric():
    rng = np.random.default_rng(9)
    a, b = _grid_sets(rng, 2, 3, 3, 8)
    b = np.vstack([b, a[:1]])   # b holds a's first vector: min is 0 both ways
    assert search.set_key(a, b, "min") == 0.0
    assert search.set_key(a, b, "meanmin") != search.set_key(b, a, "meanmin")


def test_meanmin_ranking_decided_in_float32():
    # Two one-vector sets whose distances from q differ below float32
    # resolution: float64 puts set 1 first, float32 ties them and the lower
    # id wins; Min (exact integers) keeps the float64 order.
    q = np.zeros((1, 3))
    v_far = np.array([[4000, 1002, 1]]) / 4096.0     # 2^24 d^2 = 17,004,005
    v_near = np.array([[4000, 1002, 0]]) / 4096.0    # 2^24 d^2 = 17,004,004
    d_far, d_near = math.sqrt(17_004_005) / 4096, math.sqrt(17_004_004) / 4096
    assert d_near < d_far and np.float32(d_near) == np.float32(d_far)
    X = np.vstack([v_far, v_near])
    off = np.array([0, 1, 2])
    ids, _, _ = search.bruteforce_metric(X, off, q, 2, "meanmin")
    assert ids.tolist() == [0, 1]
    ids, _, _ = search.bruteforce_metric(X, off, q, 2, "min")
    assert ids.tolist() == [1, 0]


def test_bruteforce_metric_against_sorting_scipy_values():
    rng = np.random.default_rng(10)
    sets = _grid_sets(rng, 40, 1, 9, 12)
    X = np.vstack(sets)
    off = np.concatenate([[0], np.cumsum([len(s) for s in sets])])
    Q = _grid_sets(rng, 1, 4, 4, 12)[0]
    for metric in ("meanmin", "min", "hausdorff"):
        vals = []
        for j, V in enumerate(sets):
            D = cdist(Q, V)
            v = {"meanmin": float(np.float32(D.min(axis=1).mean())), "min": D.min(),
                 "hausdorff": max(D.min(axis=1).max(), D.min(axis=0).max())}[metric]
            vals.append((v, j))
        want = [j for _, j in sorted(vals)[:7]]
        ids, _, dist = search.bruteforce_metric(X, off, Q, 7, metric)
        assert ids.tolist() == want, metric
        assert np.allclose(dist, [v for v, _ in sorted(vals)[:7]], rtol=1e-6)


@pytest.mark.parametrize("example,mistake", [("symmetry", "set_to_query"), ("precision", "mean_of_squares"),
                                             ("precision", "max_instead_of_mean")])
def test_pins_catch_plausible_meanmin_mistakes(example, mistake):
    ex = EX[example]
    Q, A = _points_for_matrix(ex["Q_to_A"], 5.0 if example == "precision" else 4.5)
    D = cdist(Q, A)
    wrong = {"set_to_query": D.min(axis=0).mean(),
             "mean_of_squares": math.sqrt((D.min(axis=1) ** 2).mean()),
             "max_instead_of_mean": D.min(axis=1).max()}[mistake]
    assert not math.isclose(wrong, ex["printed"]["d_mean_min(Q,A)"], rel_tol=1e-6)
