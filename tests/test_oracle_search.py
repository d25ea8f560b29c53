"""End-to-end pins of the oracle search (Alg. 6) and brute force (Def. 5)."""
import itertools
import math

import numpy as np
import pytest

from oracle import prng, search
from paper_2412_03301_amd import synth


def _tiny(n, lo, hi, d, seed):
    db = synth.make_database(n, lo, hi, d, n_topics=5, seed=seed)
    return db.vectors.numpy().astype(np.float64), db.offsets


def _py_hausdorff_sq(A, B):
    d2 = [[sum((float(x) - float(y)) ** 2 for x, y in zip(p, q)) for q in B] for p in A]
    return max(max(min(r) for r in d2), max(min(d2[i][j] for i in range(len(A)))
                                            for j in range(len(B))))


def test_bruteforce_exhaustive_tiny():
    X, off = _tiny(24, 1, 5, 6, seed=3)
    Q = X[off[4]:off[5]][:2] + 1.0 / 4096
    ids, h2, dist = search.bruteforce(X, off, Q, k=5)
    ref = sorted((_py_hausdorff_sq(Q, X[off[j]:off[j + 1]]), j) for j in range(24))[:5]
    assert ids.tolist() == [j for _, j in ref]
    for (r, _), v in zip(ref, h2):
        assert math.isclose(r, v, rel_tol=1e-12, abs_tol=0)
    assert np.allclose(dist, np.sqrt(h2).astype(np.float32))


@pytest.mark.parametrize("seed", [0, 1])
def test_no_filtering_reduces_to_bruteforce(seed):
    # M = 0 admits every set and T >= n keeps them all, so the cascade must
    # return exactly the brute-force top-k.
    X, off = _tiny(120, 2, 9, 16, seed=seed)
    idx = prng.projection_rows(seed, 16, 128, 3)
    ix = search.build_index(X, off, idx, 8)
    n = len(off) - 1
    for j in (0, 17, 99):
        Q = X[off[j]:off[j + 1]][::-1]
        res = search.search(ix, Q, A=3, M=0, T=n, k=10)
        ids, h2, _ = search.bruteforce(X, off, Q, 10)
        assert res["ids"].tolist() == ids.tolist()
        assert res["h2"].tolist() == h2.tolist()


def test_query_identical_to_a_set_ranks_it_first():
    X, off = _tiny(200, 3, 10, 32, seed=4)
    idx = prng.projection_rows(4, 32, 256, 4)
    ix = search.build_index(X, off, idx, 8)
    for j in (3, 50, 150):
        res = search.search(ix, ix.members(j), A=3, M=1, T=20, k=3)
        assert res["ids"][0] == j and res["h2"][0] == 0.0
        assert res["f2_scores"][0] == 0


def test_fewer_candidates_than_k():
    X, off = _tiny(30, 2, 4, 8, seed=5)
    idx = prng.projection_rows(5, 8, 128, 2)
    ix = search.build_index(X, off, idx, 4)
    res = search.search(ix, ix.members(0), A=1, M=1, T=3, k=10)
    assert len(res["ids"]) == len(res["f2_ids"]) <= 3


def test_recall_on_synthetic_workload_is_high():
    # Not a parity pin: a sanity check that the filter keeps true neighbours
    # on topic-structured data (the paper reports recall@10 above 90 %).
    db = synth.make_database(600, 8, 20, 64, n_topics=20, seed=6)
    X = db.vectors.numpy().astype(np.float64)
    idx = prng.projection_rows(6, 64, 512, 8)
    ix = search.build_index(X, db.offsets, idx, 16)
    q, qoff, _ = synth.make_subset_queries(db, 8, seed=6)
    q = q.numpy().astype(np.float64)
    rec = []
    for i in range(8):
        Q = q[qoff[i]:qoff[i + 1]]
        res = search.search(ix, Q, A=3, M=1, T=60, k=10)
        truth, _, _ = search.bruteforce(X, db.offsets, Q, 10)
        rec.append(search.recall_at_k(res["ids"], truth))
    assert np.mean(rec) >= 0.8
