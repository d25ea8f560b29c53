"""The re-rank by other set measures (Sec. 3.2: MeanMin from the query to
the set, Min distance) against the oracle, through the C ABI.

Result ids are compared exactly; Min distances (square roots of exact
integers) within 1e-5 relative, MeanMin distances within 1e-6 relative
(float64 accumulation on both sides, one float32 rounding).  The filter
layers are those of bvs_search, so F2 is the oracle's F2."""
import numpy as np
import pytest

from oracle import search
from tests.gpu_util import build_case, to_np

pytestmark = pytest.mark.gpu

TOL = {"meanmin": 1e-6, "min": 1e-5, "hausdorff": 1e-5}


@pytest.fixture(scope="module")
def tiny():
    print("[metrics] tiny workload", flush=True)
    return build_case(3000, 8, 32, 128, 40, 1024, 8, 32, 200, 12)


@pytest.fixture(scope="module")
def wide():
    """d = 384, L = 4096, queries of 1-256 vectors (query tiles past the
    staged rows are read from global memory)."""
    print("[metrics] d=384 workload, queries up to 256 vectors", flush=True)
    return build_case(1500, 5, 100, 384, 30, 4096, 16, 64, 150, 5, queries=[1, 17, 100, 64, 256])


def _check(case, metric, k=10):
    ids, dist, cnt = case.ix_gpu.search_metric(case.q, case.q_off, k, metric)
    ids, dist, cnt = to_np(ids).view(np.uint32), to_np(dist), to_np(cnt)
    p = case.params
    for i in range(len(case.q_off) - 1):
        r = search.search_metric(case.ix_oracle, case.query(i), A=p.access_lists, M=p.min_count, T=p.top_t, k=k,
                                 metric=metric)
        c = len(r["ids"])
        assert cnt[i] == c
        assert ids[i, :c].astype(np.int64).tolist() == r["ids"].tolist(), (metric, i)
        np.testing.assert_allclose(dist[i, :c], r["dist"], rtol=TOL[metric], atol=0)
        assert (ids[i, c:] == 0xFFFFFFFF).all() and np.isinf(dist[i, c:]).all()


@pytest.mark.parametrize("metric", ["meanmin", "min"])
def test_search_metric_tiny(tiny, metric):
    _check(tiny, metric)


@pytest.mark.parametrize("metric", ["meanmin", "min"])
def test_search_metric_wide_queries(wide, metric):
    _check(wide, metric)


def test_search_metric_hausdorff_equals_search(tiny):
    a = [to_np(t) for t in tiny.ix_gpu.search(tiny.q, tiny.q_off, 10)]
    b = [to_np(t) for t in tiny.ix_gpu.search_metric(tiny.q, tiny.q_off, 10, "hausdorff")]
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))


@pytest.mark.parametrize("metric", ["meanmin", "min", "hausdorff"])
def test_bruteforce_metric(tiny, metric):
    nq = 4
    off = tiny.q_off[:nq + 1]
    q = tiny.q[:int(off[-1])].contiguous()
    ids, dist, cnt = tiny.ix_gpu.bruteforce_metric(q, off, 10, metric)
    ids, dist = to_np(ids).view(np.uint32), to_np(dist)
    for i in range(nq):
        r_ids, _, r_dist = search.bruteforce_metric(tiny.X, tiny.db.offsets, tiny.query(i), 10, metric)
        assert ids[i].astype(np.int64).tolist() == r_ids.tolist(), (metric, i)
        np.testing.assert_allclose(dist[i], r_dist, rtol=TOL[metric], atol=0)


@pytest.mark.parametrize("name,n_q", [("tiny", 7), ("wide", 1), ("wide", 3), ("wide", 4), ("wide", 5)])
def test_bruteforce_query_tiles_with_ragged_tail(name, n_q, request):
    # several queries share each database set's registers (tiles of 4 small
    # queries, or of 2 with rows past the staged ones read from global
    # memory); the last tile of queries is partly empty; a batch holding a
    # query of more than 128 vectors takes one query per workgroup
    case = request.getfixturevalue(name)
    off = case.q_off[:n_q + 1]
    q = case.q[:int(off[-1])].contiguous()
    for metric in ("hausdorff", "meanmin"):
        ids, dist, cnt = case.ix_gpu.bruteforce_metric(q, off, 10, metric)
        ids, dist = to_np(ids).view(np.uint32), to_np(dist)
        for i in range(n_q):
            r_ids, _, r_dist = search.bruteforce_metric(case.X, case.db.offsets, case.query(i), 10, metric)
            assert ids[i].astype(np.int64).tolist() == r_ids.tolist(), (metric, i)
            np.testing.assert_allclose(dist[i], r_dist, rtol=TOL[metric], atol=0)
