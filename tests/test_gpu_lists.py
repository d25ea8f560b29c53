"""The inverted lists (Def. 9, Alg. 4) and the first filter layer read from
them, against the oracle, through the C ABI.

Each list must hold exactly the sets with a nonzero count at its position,
in non-increasing count order (equal counts in any order, as Alg. 4 sorts
by count only), with the count-class boundaries right; the candidate lists
F2 of searches whose first layer comes from the lists must equal the
oracle's bit for bit, for A = 1..3 and M = 1, 2, 3."""
import numpy as np
import pytest

from oracle import index as oindex
from oracle import search
from tests.gpu_util import build_case, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    print("[lists] workload: 2,000 sets, L = 1024", flush=True)
    c = build_case(2000, 8, 32, 128, 40, 1024, 8, 32, 200, 8)
    c.ix_gpu.attach_lists()
    return c


def test_lists_hold_each_positions_sets_by_decreasing_count(case):
    cum, start, ids = (to_np(t) for t in case.ix_gpu.lists_views())
    C = case.ix_oracle.C                       # [n, L]
    n, L = C.shape
    assert start[0] == 0 and start[-1] == len(ids) == int((C > 0).sum())
    lists = oindex.build_inverted_index(C)     # literal Alg. 4 (every set, count 0 included)
    for p in range(L):
        got = ids[start[p]:start[p + 1]].astype(np.int64)
        want = [(j, c) for j, c in lists[p] if c >= 1]
        assert sorted(got.tolist()) == sorted(j for j, _ in want), p
        counts = C[got, p]
        assert (np.diff(counts) <= 0).all(), p
        for c in range(1, 257):
            assert cum[p, c] == int((C[:, p] >= c).sum()), (p, c)
        assert cum[p, 0] == cum[p, 1]


@pytest.mark.parametrize("A,M", [(1, 1), (2, 1), (3, 1), (3, 2), (2, 3)])
def test_candidates_from_lists_match_oracle(case, A, M):
    ix = case.ix_gpu
    T = case.params.top_t
    try:
        ix.set_search_params(A, M, T)
        ix.set_first_layer("lists")
        ids, sc, cnt = ix.candidates(case.q, case.q_off)
    finally:
        ix.set_first_layer("bitmaps")
        ix.set_search_params(3, 1, T)
    ids, sc, cnt = to_np(ids).view(np.uint32), to_np(sc).view(np.uint16), to_np(cnt)
    for i in range(len(case.q_off) - 1):
        r = search.search(case.ix_oracle, case.query(i), A=A, M=M, T=T, k=10)
        c = len(r["f2_ids"])
        assert cnt[i] == c
        assert ids[i, :c].astype(np.int64).tolist() == r["f2_ids"].tolist()
        assert sc[i, :c].astype(np.int64).tolist() == r["f2_scores"].tolist()


def test_search_with_lists_equals_bitmaps(case):
    ix = case.ix_gpu
    a = [to_np(t) for t in ix.search(case.q, case.q_off, 10)]
    ix.set_first_layer("lists")
    try:
        b = [to_np(t) for t in ix.search(case.q, case.q_off, 10)]
    finally:
        ix.set_first_layer("bitmaps")
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))


def test_lists_mode_needs_attached_lists():
    from paper_2412_03301_amd import bvs
    c = build_case(300, 3, 20, 64, 8, 512, 4, 16, 60, 2)
    with pytest.raises(bvs.BvsError) as e:
        c.ix_gpu.set_first_layer("lists")
    assert e.value.status == bvs.BVS_ESTATE
