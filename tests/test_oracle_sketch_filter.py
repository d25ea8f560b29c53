"""Pins of the oracle's sketches and filters (Defs. 8-10, Algs. 3-6)."""
import numpy as np
import pytest
import torch

from oracle import filter as flt
from oracle import flyhash, index, prng, search, sketch
from paper_2412_03301_amd import synth


@pytest.fixture(scope="module")
def small():
    torch.manual_seed(0)
    db = synth.make_database(300, 3, 12, 32, n_topics=6, seed=11)
    X = db.vectors.numpy().astype(np.float64)
    idx = prng.projection_rows(9, 32, 256, 4)
    ix = search.build_index(X, db.offsets, idx, 8)
    return db, ix


def test_count_and_binary_bloom_invariants(small):
    db, ix = small
    m = np.diff(db.offsets)
    assert (ix.C.sum(axis=1) == 8 * m).all()          # sum C = k_wta * m
    assert (ix.B == (ix.C > 0)).all()                  # B = [C > 0]
    assert (ix.C <= m[:, None]).all()
    for j in range(ix.n_sets):                         # no false negatives
        H = ix.H[db.offsets[j]:db.offsets[j + 1]]
        assert not (H & ~ix.B[j]).any()


def test_singleton_set_sketch_is_its_code():
    rng = np.random.default_rng(0)
    idx = prng.projection_rows(1, 16, 128, 3)
    X = np.round(rng.standard_normal((5, 16)) * 256) / 4096
    H = flyhash.codes(X, idx, 6)
    off = np.arange(6)
    assert (sketch.count_bloom(H, off) == H).all()
    assert (sketch.binary_bloom(H, off) == H).all()


def test_count_bloom_against_bitwise_loop():
    rng = np.random.default_rng(1)
    H = rng.random((20, 40)) < 0.2
    off = np.array([0, 3, 4, 12, 20])
    C = sketch.count_bloom(H, off)
    for j in range(4):
        for i in range(40):
            assert C[j, i] == sum(int(H[r, i]) for r in range(off[j], off[j + 1]))


def test_top_positions_ties_and_order():
    C_Q = np.array([2, 5, 5, 1, 5, 0, 7])
    assert flt.top_positions(C_Q, 1).tolist() == [6]
    assert flt.top_positions(C_Q, 3).tolist() == [6, 1, 2]
    assert flt.top_positions(C_Q, 5).tolist() == [6, 1, 2, 4, 0]


def test_min_count_zero_admits_every_set(small):
    _, ix = small
    P = np.array([0, 1, 2])
    assert flt.first_filter(ix.C, P, 0).all()


def test_subset_query_keeps_its_source(small):
    db, ix = small
    for j in range(0, ix.n_sets, 37):
        Q = ix.members(j)[::2]
        res = search.search(ix, Q, A=3, M=1, T=5, k=3)
        assert res["member"][j]
        # S_Q is contained in B_src, so the Hamming distance is the size gap.
        assert res["scores"][j] == ix.B[j].sum() - res["S_Q"].sum()
        assert flt.hamming(ix.B[j], ix.B[j:j + 1])[0] == 0


@pytest.mark.parametrize("M", [0, 1, 2, 3])
def test_dense_first_filter_equals_inverted_lists(small, M):
    _, ix = small
    lists = index.build_inverted_index(ix.C)
    rng = np.random.default_rng(M)
    for _ in range(4):
        P = rng.choice(ix.C.shape[1], size=3, replace=False)
        dense = set(np.flatnonzero(flt.first_filter(ix.C, P, M)).tolist())
        assert dense == index.first_filter_lists(lists, P, M)


@pytest.mark.parametrize("T", [1, 7, 50, 1000])
def test_second_filter_equals_literal_heap(small, T):
    db, ix = small
    Q = ix.members(5)
    res = search.search(ix, Q, A=3, M=1, T=T, k=3)
    F1 = np.flatnonzero(res["member"])
    heap = index.second_filter_heap(F1.tolist(), res["S_Q"], ix.B, T)
    assert [i for _, i in heap] == res["f2_ids"].tolist()
    assert [d for d, _ in heap] == res["f2_scores"].tolist()


def test_second_filter_with_many_ties():
    member = np.ones(10, bool)
    scores = np.array([3, 1, 3, 3, 0, 3, 1, 3, 3, 2])
    ids, sc = flt.second_filter(member, scores, 6)
    assert ids.tolist() == [4, 1, 6, 9, 0, 2]
    assert sc.tolist() == [0, 1, 1, 2, 3, 3]
    member[1] = False
    ids, _ = flt.second_filter(member, scores, 3)
    assert ids.tolist() == [4, 6, 9]
