"""Parity of the HIP path against the CPU oracle, through the C ABI.

Codes, sketches, query sketches, candidate lists and result ids must be
bit-exact; squared Hausdorff distances (2^24-scaled integers) must be equal,
and reported distances within 1e-5 relative of the float64 oracle."""
import numpy as np
import pytest
import torch

from oracle import filter as flt
from oracle import flyhash, search
from tests.gpu_util import build_case, oracle_query_codes, to_np

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5


def _print_case(name):
    print(f"[parity] {name}", flush=True)


@pytest.fixture(scope="module")
def tiny():
    """5,000 sets of 8-32 vectors, d = 128, L = 1024, s = 8, k = 32, T = 200."""
    _print_case("tiny workload")
    return build_case(5000, 8, 32, 128, 50, 1024, 8, 32, 200, 16)


def test_encode_bit_exact(tiny):
    codes = to_np(tiny.ix_gpu.encode(tiny.db.vectors.cuda())).view(np.uint64)
    ref = flyhash.pack(tiny.ix_oracle.H)
    assert codes.shape == ref.shape
    assert np.array_equal(codes, ref)


def test_sketches_bit_exact(tiny):
    cnt, bits = tiny.ix_gpu.sketch_views()
    n = tiny.ix_oracle.n_sets
    cnt = to_np(cnt)
    assert np.array_equal(cnt[:, :n].T.astype(np.int64), tiny.ix_oracle.C)
    assert not cnt[:, n:].any()
    b = to_np(bits).view(np.uint64)              # [L/128, ld, 2]
    words = b.transpose(1, 0, 2).reshape(b.shape[1], -1)   # [ld, L/64]
    assert np.array_equal(words[:n], flyhash.pack(tiny.ix_oracle.B))
    assert not words[n:].any()


def test_query_sketch_bit_exact(tiny):
    cq, sq, pos = tiny.ix_gpu.query_sketch(tiny.q, tiny.q_off)
    cq, sq, pos = to_np(cq).view(np.uint16), to_np(sq).view(np.uint64), to_np(pos)
    for i in range(len(tiny.q_off) - 1):
        HQ = oracle_query_codes(tiny, i)
        C_Q, S_Q = flt.query_sketches(HQ)
        assert np.array_equal(cq[i].astype(np.int64), C_Q)
        assert np.array_equal(sq[i], flyhash.pack(S_Q[None])[0])
        assert pos[i].tolist() == flt.top_positions(C_Q, 3).tolist()


def _oracle_results(case, A, M, T, k):
    key = (A, M, T, k)
    cache = case.__dict__.setdefault("_res", {})
    if key not in cache:
        cache[key] = [search.search(case.ix_oracle, case.query(i), A=A, M=M, T=T, k=k)
                      for i in range(len(case.q_off) - 1)]
    return cache[key]


def _check_candidates(case, res, T):
    ids, sc, cnt = case.ix_gpu.candidates(case.q, case.q_off)
    ids, sc, cnt = to_np(ids).view(np.uint32), to_np(sc).view(np.uint16), to_np(cnt)
    for i, r in enumerate(res):
        c = len(r["f2_ids"])
        assert cnt[i] == c
        assert ids[i, :c].astype(np.int64).tolist() == r["f2_ids"].tolist()
        assert sc[i, :c].astype(np.int64).tolist() == r["f2_scores"].tolist()
        assert (ids[i, c:] == 0xFFFFFFFF).all() and (sc[i, c:] == 0xFFFF).all()


def _check_search(case, res, k):
    ids, dist, cnt = case.ix_gpu.search(case.q, case.q_off, k)
    ids, dist, cnt = to_np(ids).view(np.uint32), to_np(dist), to_np(cnt)
    for i, r in enumerate(res):
        c = len(r["ids"])
        assert cnt[i] == c
        assert ids[i, :c].astype(np.int64).tolist() == r["ids"].tolist()
        ref = np.sqrt(r["h2"])
        np.testing.assert_allclose(dist[i, :c], ref, rtol=REL_TOL, atol=0)
        assert (ids[i, c:] == 0xFFFFFFFF).all() and np.isinf(dist[i, c:]).all()


def test_candidates_bit_exact(tiny):
    res = _oracle_results(tiny, 3, 1, 200, 10)
    _check_candidates(tiny, res, 200)


def test_candidates_with_large_ties():
    """Candidate lists stay bit-exact when many candidates share a score:
    400, 300 and 100 exact copies of three sets (ties at the smallest score
    larger than T = 200, about T and below it, broken by set id) among
    1,200 other sets; the queries are the three copied sets and four other
    sets."""
    from oracle import prng
    from paper_2412_03301_amd import bvs
    _print_case("score ties of 400, 300 and 100 candidates")
    rng = np.random.default_rng(5)
    d = 128

    def grid(x):
        x = x / np.linalg.norm(x, axis=1, keepdims=True)
        return (np.rint(x * 4096) / 4096).astype(np.float32)

    bases = [grid(rng.normal(size=(int(rng.integers(4, 16)), d))) for _ in range(3)]
    sets = []
    for b, n in zip(bases, (400, 300, 100)):
        sets += [b] * n
    sets += [grid(rng.normal(size=(int(rng.integers(4, 16)), d))) for _ in range(1200)]
    order = rng.permutation(len(sets))
    sets = [sets[i] for i in order]
    off = np.concatenate([[0], np.cumsum([len(x) for x in sets])]).astype(np.int64)
    X = np.concatenate(sets)
    qs = bases + [sets[i] for i in (3, 500, 1000, 1500)]
    q_off = np.concatenate([[0], np.cumsum([len(x) for x in qs])]).astype(np.int64)
    Q = np.concatenate(qs)
    T = 200
    p = bvs.Params.make(dim=d, code_bits=1024, fan_in=8, wta_k=32, access_lists=3, min_count=1, top_t=T, seed=4)
    ix_g = bvs.Index(p, torch.from_numpy(X).cuda(), off)
    ix_o = search.build_index(X.astype(np.float64), off, prng.projection_rows(4, d, 1024, 8), 32)
    ids, sc, cnt = ix_g.candidates(torch.from_numpy(Q).cuda().contiguous(), q_off)
    ids, sc, cnt = to_np(ids).view(np.uint32), to_np(sc).view(np.uint16), to_np(cnt)
    for i in range(len(q_off) - 1):
        r = search.search(ix_o, Q[q_off[i]:q_off[i + 1]].astype(np.float64), A=3, M=1, T=T, k=10)
        c = len(r["f2_ids"])
        assert cnt[i] == c
        assert ids[i, :c].astype(np.int64).tolist() == r["f2_ids"].tolist()
        assert sc[i, :c].astype(np.int64).tolist() == r["f2_scores"].tolist()
        if i < 3:
            assert (r["f2_scores"][: min(T, (400, 300, 100)[i])] == 0).all()


def test_search_matches_oracle(tiny):
    res = _oracle_results(tiny, 3, 1, 200, 10)
    _check_search(tiny, res, 10)


@pytest.mark.parametrize("env,fallback", [({}, False), ({"BVS_SELECT": "dense"}, True),
                                          ({"BVS_APPEND_CAP": "8"}, True), ({"BVS_APPEND_CAP": "300"}, None),
                                          ({"BVS_FILTER": "dense"}, False),
                                          ({"BVS_FILTER": "dense", "BVS_APPEND_CAP": "8"}, True)])
def test_selection_paths_agree(tiny, monkeypatch, env, fallback):
    from paper_2412_03301_amd import bvs
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    res = _oracle_results(tiny, 3, 1, 200, 10)
    bvs.profile_enable(True)
    _check_candidates(tiny, res, 200)
    _check_search(tiny, res, 10)
    used = bvs.profile_read()["fallback"][1] > 0
    bvs.profile_enable(False)
    if fallback is not None:
        assert used == fallback


def test_screen_keeps_results(tiny, monkeypatch):
    """The high-plane screen only drops candidates that cannot be in the
    top-k: results with and without it are identical, and it does reject
    some candidates."""
    from paper_2412_03301_amd import bvs
    runs = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("BVS_SCREEN", flag)
        bvs.profile_enable(False, counters=True)
        out = [to_np(t) for t in tiny.ix_gpu.search(tiny.q, tiny.q_off, 10)]
        runs[flag] = (out, bvs.profile_counters())
        bvs.profile_enable(False)
    for x, y in zip(runs["1"][0], runs["0"][0]):
        assert np.array_equal(x, y)
    on, off = runs["1"][1], runs["0"][1]
    assert 0 < on["rerank_screened"] <= on["rerank_abandoned"]
    assert on["rerank_screen_vectors"] > 0
    assert off["rerank_screened"] == 0 and off["rerank_screen_vectors"] == 0
    assert on["rerank_candidates"] == off["rerank_candidates"]


def _near_duplicate_case():
    """300 clusters of 12 near-copies of one base set (copies differ by
    noise of norm 0.004 per vector, so Hausdorff distances within a cluster
    are about 0.006) and 8 queries that are noisy copies of a cluster: the
    10th distance is far below 0.02, the regime where the screen's bound is
    small against the residual terms."""
    from oracle import prng
    from paper_2412_03301_amd import bvs
    rng = np.random.default_rng(11)
    d, n_cl, copies = 128, 300, 12

    def grid(x):
        x = x / np.linalg.norm(x, axis=1, keepdims=True)
        return (np.rint(x * 4096) / 4096).astype(np.float32)

    sets, bases = [], []
    for c in range(n_cl):
        base = rng.normal(size=(int(rng.integers(3, 20)), d))
        base /= np.linalg.norm(base, axis=1, keepdims=True)
        bases.append(base)
        for _ in range(copies):
            sets.append(grid(base + rng.normal(size=base.shape) * 0.004 / np.sqrt(d)))
    off = np.concatenate([[0], np.cumsum([len(x) for x in sets])]).astype(np.int64)
    X = np.concatenate(sets)
    qs = [grid(bases[c] + rng.normal(size=bases[c].shape) * 0.004 / np.sqrt(d)) for c in range(0, n_cl, 37)]
    q_off = np.concatenate([[0], np.cumsum([len(x) for x in qs])]).astype(np.int64)
    Q = np.concatenate(qs)
    p = bvs.Params.make(dim=d, code_bits=1024, fan_in=8, wta_k=32, access_lists=3, min_count=1, top_t=200, seed=2)
    ix_g = bvs.Index(p, torch.from_numpy(X).cuda(), off)
    ix_o = search.build_index(X.astype(np.float64), off, prng.projection_rows(2, d, 1024, 8), 32)
    return ix_g, ix_o, torch.from_numpy(Q).cuda().contiguous(), Q.astype(np.float64), q_off


def test_screen_near_duplicates(monkeypatch):
    """With a 10th distance below 0.02 the screen still keeps every result:
    screen on and off agree with each other and with the oracle."""
    from paper_2412_03301_amd import bvs
    _print_case("near-duplicate clusters, screen on and off")
    ix_g, ix_o, q, Q, q_off = _near_duplicate_case()
    runs = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("BVS_SCREEN", flag)
        bvs.profile_enable(False, counters=True)
        runs[flag] = ([to_np(t) for t in ix_g.search(q, q_off, 10)], bvs.profile_counters())
        bvs.profile_enable(False)
    for x, y in zip(runs["1"][0], runs["0"][0]):
        assert np.array_equal(x, y)
    assert runs["1"][1]["rerank_screen_vectors"] > 0
    ids, dist, cnt = runs["1"][0]
    ids = ids.view(np.uint32)
    for i in range(len(q_off) - 1):
        r = search.search(ix_o, Q[q_off[i]:q_off[i + 1]], A=3, M=1, T=200, k=10)
        assert np.sqrt(r["h2"][-1]) < 0.02
        assert ids[i].astype(np.int64).tolist() == r["ids"].tolist()
        np.testing.assert_allclose(dist[i], np.sqrt(r["h2"]), rtol=REL_TOL, atol=0)


def test_hausdorff_all_exact(tiny):
    h2 = to_np(tiny.ix_gpu.hausdorff_all(tiny.q, tiny.q_off)).astype(np.int64)
    for i in range(4):
        ref = search.all_hausdorff_sq(tiny.X, tiny.db.offsets, tiny.query(i)) * 2.0 ** 24
        assert np.array_equal(h2[i], ref.astype(np.int64))


def test_bruteforce_matches_oracle(tiny):
    ids, dist, cnt = tiny.ix_gpu.bruteforce(tiny.q, tiny.q_off, 10)
    ids, dist, cnt = to_np(ids).view(np.uint32), to_np(dist), to_np(cnt)
    for i in range(len(tiny.q_off) - 1):
        rid, rh2, _ = search.bruteforce(tiny.X, tiny.db.offsets, tiny.query(i), 10)
        assert cnt[i] == 10
        assert ids[i].astype(np.int64).tolist() == rid.tolist()
        np.testing.assert_allclose(dist[i], np.sqrt(rh2), rtol=REL_TOL, atol=0)


def test_repeatable_and_batch_independent(tiny):
    a = [to_np(t) for t in tiny.ix_gpu.search(tiny.q, tiny.q_off, 10)]
    b = [to_np(t) for t in tiny.ix_gpu.search(tiny.q, tiny.q_off, 10)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # each query alone gives the same answer as inside the batch
    for i in (0, 7, 15):
        o0, o1 = tiny.q_off[i], tiny.q_off[i + 1]
        qi = tiny.q[o0:o1].contiguous()
        ids, dist, cnt = [to_np(t) for t in tiny.ix_gpu.search(qi, [0, o1 - o0], 10)]
        assert np.array_equal(ids[0], a[0][i]) and np.array_equal(dist[0], a[1][i])


def test_invalid_query_values_are_rejected(tiny):
    from paper_2412_03301_amd import bvs
    bad = tiny.q[:5].clone()
    bad[2, 3] += 1e-4                       # off the 2^-12 grid
    with pytest.raises(bvs.BvsError) as e:
        tiny.ix_gpu.search(bad.contiguous(), [0, 5], 10)
    assert e.value.status == bvs.BVS_ERANGE
    big = tiny.q[:5].clone() * 4.0          # on the grid, but norm 4 and |x| may exceed 1
    with pytest.raises(bvs.BvsError):
        tiny.ix_gpu.search(big.contiguous(), [0, 5], 10)
    ids, _, _ = tiny.ix_gpu.search(tiny.q, tiny.q_off, 10)   # still usable afterwards
    assert ids.shape[0] == 16


# ------------------------------------------------------------------ variants
VARIANTS = {
    # name: (n_sets, lo, hi, d, topics, L, s, wta_k, T, n_q, A, M, queries)
    "min_count_0": (700, 3, 12, 64, 8, 512, 4, 16, 50, 6, 3, 0, "subset"),
    "min_count_2": (700, 3, 12, 64, 8, 512, 4, 16, 50, 6, 3, 2, "subset"),
    "all_candidates": (300, 1, 6, 64, 5, 256, 4, 8, 4096, 5, 1, 0, "subset"),
    "singletons": (900, 1, 1, 32, 10, 256, 3, 8, 40, 8, 2, 1, "subset"),
    "ragged_d100_L2048": (1333, 2, 40, 100, 12, 2048, 6, 40, 300, 7, 8, 1, "subset"),
    "d384_L4096": (1100, 5, 100, 384, 20, 4096, 16, 64, 500, 5, 3, 1, "subset"),
    "d768_fresh_queries": (600, 5, 60, 768, 10, 4096, 16, 64, 200, 6, 3, 1, 48),
    "big_queries": (500, 2, 30, 128, 6, 1024, 8, 32, 100, 4, 3, 1, 128),
    "sampled_cutoff_30k": (30000, 2, 16, 64, 300, 512, 4, 16, 100, 6, 3, 1, "subset"),
    # more queries than one pass of the bit-sliced filter's waves
    "many_queries": (2600, 2, 20, 64, 40, 1024, 4, 24, 60, 300, 3, 1, "subset"),
    # long and short query sketches in one call: both bit-sliced instances
    "mixed_sketches": (2000, 2, 20, 64, 30, 1024, 4, 32, 60, 70, 3, 1,
                       [60, 1, 45, 2, 3, 1, 2] * 10),
    # d = 768 with a 100-vector query: the exact re-rank stages only part of
    # the query in LDS while the screen stages all of its high plane
    "d768_long_queries": (400, 5, 60, 768, 8, 4096, 16, 64, 150, 3, 3, 1, [100, 5, 70]),
}


@pytest.fixture(scope="module", params=sorted(VARIANTS))
def variant(request):
    n, lo, hi, d, top, L, s, k, T, nq, A, M, qk = VARIANTS[request.param]
    _print_case(f"variant {request.param}")
    return build_case(n, lo, hi, d, top, L, s, k, T, nq, A=A, M=M, seed=3, queries=qk), (A, M, T)


@pytest.mark.parametrize("filt", ["default", "dense", "sparse"])
def test_variant_pipeline(variant, filt, monkeypatch):
    if filt != "default":
        monkeypatch.setenv("BVS_FILTER", filt)
    case, (A, M, T) = variant
    k = min(10, T)
    assert np.array_equal(to_np(case.ix_gpu.encode(case.db.vectors.cuda())).view(np.uint64),
                          flyhash.pack(case.ix_oracle.H))
    res = _oracle_results(case, A, M, T, k)
    _check_candidates(case, res, T)
    _check_search(case, res, k)
