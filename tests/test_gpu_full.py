"""The full-scan search (Alg. 2) against the oracle, through the C ABI.

Haus^H scores of every (query, set) pair and the candidate lists F are
compared bit for bit; result ids exactly, distances within 1e-5 relative."""
import numpy as np
import pytest

from oracle import biovss
from tests.gpu_util import build_case, to_np

pytestmark = pytest.mark.gpu


def _attached(case):
    if not getattr(case, "_codes_attached", False):
        case.ix_gpu.attach_codes()
        case._codes_attached = True
    return case


@pytest.fixture(scope="module")
def tiny():
    """2,000 sets of 8-32 vectors, d = 128, L = 1024, s = 8, k = 32, c = 200."""
    print("[full] tiny workload", flush=True)
    return _attached(build_case(2000, 8, 32, 128, 40, 1024, 8, 32, 200, 8))


@pytest.fixture(scope="module")
def wide():
    """d = 384, L = 4096, s = 16, k = 64, sets of 5-100 vectors, queries of
    1-256 vectors (one to four groups of 64 query vectors)."""
    print("[full] d=384 workload, queries up to 256 vectors", flush=True)
    return _attached(build_case(500, 5, 100, 384, 20, 4096, 16, 64, 100, 6,
                                queries=[1, 40, 64, 65, 190, 256]))


def _oracle(case, i):
    cache = case.__dict__.setdefault("_full", {})
    if i not in cache:
        cache[i] = biovss.search_full(case.ix_oracle, case.query(i), c=case.params.top_t, k=10)
    return cache[i]


def _n_q(case):
    return len(case.q_off) - 1


@pytest.mark.parametrize("name", ["tiny", "wide"])
def test_scores_bit_exact(name, request):
    case = request.getfixturevalue(name)
    sc = to_np(case.ix_gpu.full_scores(case.q, case.q_off)).view(np.uint16)
    for i in range(_n_q(case)):
        assert np.array_equal(sc[i].astype(np.int64), _oracle(case, i)["scores"]), i


@pytest.mark.parametrize("name", ["tiny", "wide"])
def test_candidates_bit_exact(name, request):
    case = request.getfixturevalue(name)
    ids, sc, cnt = case.ix_gpu.full_candidates(case.q, case.q_off)
    ids, sc, cnt = to_np(ids).view(np.uint32), to_np(sc).view(np.uint16), to_np(cnt)
    T = case.params.top_t
    for i in range(_n_q(case)):
        r = _oracle(case, i)
        c = len(r["f_ids"])
        assert c == min(T, case.ix_oracle.n_sets) and cnt[i] == c
        assert ids[i, :c].astype(np.int64).tolist() == r["f_ids"].tolist()
        assert sc[i, :c].astype(np.int64).tolist() == r["f_scores"].tolist()


@pytest.mark.parametrize("name", ["tiny", "wide"])
def test_results(name, request):
    case = request.getfixturevalue(name)
    ids, dist, cnt = case.ix_gpu.search_full(case.q, case.q_off, 10)
    ids, dist, cnt = to_np(ids).view(np.uint32), to_np(dist), to_np(cnt)
    for i in range(_n_q(case)):
        r = _oracle(case, i)
        assert cnt[i] == len(r["ids"]) == 10
        assert ids[i].astype(np.int64).tolist() == r["ids"].tolist()
        np.testing.assert_allclose(dist[i], np.sqrt(r["h2"]), rtol=1e-5, atol=0)


def test_full_scan_needs_attached_codes():
    from paper_2412_03301_amd import bvs
    case = build_case(300, 3, 20, 64, 8, 512, 4, 16, 60, 2)
    with pytest.raises(bvs.BvsError) as e:
        case.ix_gpu.search_full(case.q, case.q_off, 10)
    assert e.value.status == bvs.BVS_ESTATE


def test_scores_of_packed_small_queries(tiny):
    # twelve one-vector queries and then three larger ones: packs of eight
    # queries, of several queries sharing a group of 64 slots, and a query
    # straddling two groups
    sizes = [1] * 12 + [30, 50, 70]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    rows = np.concatenate([np.arange(12), np.arange(12, 12 + 150) % int(tiny.q_off[-1])])
    q = tiny.q[rows].contiguous()
    sc = to_np(tiny.ix_gpu.full_scores(q, off)).view(np.uint16)
    qn = q.cpu().numpy().astype(np.float64)
    from oracle import flyhash
    for i in range(len(sizes)):
        Q = qn[off[i]:off[i + 1]]
        HQ = flyhash.codes(Q, tiny.ix_oracle.idx, tiny.ix_oracle.wta_k)
        assert np.array_equal(sc[i].astype(np.int64), biovss.full_scores(tiny.ix_oracle, HQ)), i
