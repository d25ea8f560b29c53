"""Batched search: the whole cascade for many query sets of uneven size
with one persistent re-rank launch, replayed from a hipGraph, its shape
chosen by the autotuner.  Parity bar: results bit-identical to per-call
search (which the oracle pins) for every shape, replay and selection path,
and equal to the oracle directly on query sets of 1 to 256 vectors."""
import numpy as np
import pytest
import torch

from oracle import search
from paper_2412_03301_amd import synth
from tests.gpu_util import build_case, to_np

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5
# sizes spanning every query-tile edge up to the 256-vector limit
SIZES = [1, 2, 15, 16, 17, 31, 33, 64, 65, 100, 127, 128, 129, 144, 145, 160, 200, 255, 256, 3, 7, 48, 90, 250]
T, K = 300, 10


def _say(msg):
    print(f"[batch] {msg}", flush=True)


@pytest.fixture(scope="module")
def mixed():
    """1,500 sets of 5-60 vectors at d = 384 (L = 2048, s = 8, k_wta = 32),
    24 fresh-entity queries of the sizes above."""
    _say("building mixed-size workload d=384")
    return build_case(1500, 5, 60, 384, 12, 2048, 8, 32, T, len(SIZES), seed=5, queries=SIZES)


@pytest.fixture(scope="module")
def oracle_res(mixed):
    _say("oracle search over 24 queries")
    return [search.search(mixed.ix_oracle, mixed.query(i), A=3, M=1, T=T, k=K) for i in range(len(SIZES))]


@pytest.fixture(scope="module")
def per_call(mixed):
    return [to_np(t) for t in mixed.ix_gpu.search(mixed.q, mixed.q_off, K)]


def _check_oracle(res, ids, dist, cnt):
    ids = ids.view(np.uint32)
    for i, r in enumerate(res):
        c = len(r["ids"])
        assert cnt[i] == c
        assert ids[i, :c].astype(np.int64).tolist() == r["ids"].tolist(), f"query {i}"
        np.testing.assert_allclose(dist[i, :c], np.sqrt(r["h2"]), rtol=REL_TOL, atol=0)


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_per_call_search_big_queries_matches_oracle(mixed, oracle_res, per_call):
    _check_oracle(oracle_res, *per_call)


def test_bruteforce_big_queries_matches_oracle(mixed):
    sel = [SIZES.index(s) for s in (129, 256, 1, 200)]
    for i in sel:
        o0, o1 = mixed.q_off[i], mixed.q_off[i + 1]
        ids, dist, cnt = [to_np(t) for t in mixed.ix_gpu.bruteforce(mixed.q[o0:o1].contiguous(), [0, o1 - o0], K)]
        rid, rh2, _ = search.bruteforce(mixed.X, mixed.db.offsets, mixed.query(i), K)
        assert ids[0].view(np.uint32).astype(np.int64).tolist() == rid.tolist()
        np.testing.assert_allclose(dist[0], np.sqrt(rh2), rtol=REL_TOL, atol=0)


def test_bruteforce_grouping_matches_single_queries(mixed):
    """One brute-force call over all 24 queries groups them by size (8, 4, 2
    and 1 per pass over the database, padded tiles included); every query's
    top-k equals that of a call holding it alone (whose grouping differs)."""
    _say("brute force: all queries at once against one call per query")
    ids, dist, cnt = [to_np(t) for t in mixed.ix_gpu.bruteforce(mixed.q, mixed.q_off, K)]
    for i in range(len(SIZES)):
        o0, o1 = mixed.q_off[i], mixed.q_off[i + 1]
        i1, d1, c1 = [to_np(t) for t in mixed.ix_gpu.bruteforce(mixed.q[o0:o1].contiguous(), [0, o1 - o0], K)]
        assert cnt[i] == c1[0], f"query {i} ({SIZES[i]} vectors)"
        assert np.array_equal(ids[i], i1[0]), f"query {i} ({SIZES[i]} vectors)"
        assert np.array_equal(dist[i], d1[0]), f"query {i} ({SIZES[i]} vectors)"


@pytest.mark.parametrize("rows,waves,graph", [(16, 2, True), (32, 4, True), (64, 8, False), (128, 4, True),
                                              (144, 2, False), (48, 8, True)])
def test_batch_shapes_match_per_call(mixed, per_call, oracle_res, rows, waves, graph):
    from paper_2412_03301_amd import bvs
    _say(f"shape lds_rows={rows} waves={waves} graph={graph}")
    b = bvs.Batch(mixed.ix_gpu, mixed.q, mixed.q_off, K, lds_rows=rows, waves=waves, graph=graph)
    info = b.info()
    assert (info["lds_rows"], info["waves"], info["graph"]) == (rows, waves, graph)
    assert info["blocks"] > 0 and not info["tried"]
    out = [to_np(t) for t in b.run()]
    _same(out, per_call)
    _check_oracle(oracle_res, *out)
    b.close()


@pytest.mark.parametrize("graph", [True, False])
def test_batch_phase_sequence_matches_per_call(mixed, per_call, oracle_res, graph):
    from paper_2412_03301_amd import bvs
    _say(f"phase sequence by size class, graph={graph}")
    b = bvs.Batch(mixed.ix_gpu, mixed.q, mixed.q_off, K, graph=graph, phases=True)
    info = b.info()
    assert (info["lds_rows"], info["waves"], info["blocks"], info["graph"]) == (0, 0, 0, graph)
    assert not info["tried"]
    for _ in range(2):   # a replay sees the device state of the previous one
        out = [to_np(t) for t in b.run()]
        _same(out, per_call)
    _check_oracle(oracle_res, *out)
    b.close()


def test_graph_replays_with_eager_work_between(mixed, per_call):
    from paper_2412_03301_amd import bvs
    _say("graph replays")
    q = mixed.q.clone()
    b = bvs.Batch(mixed.ix_gpu, q, mixed.q_off, K, lds_rows=32, waves=4, graph=True)
    for rep in range(3):
        _same([to_np(t) for t in b.run()], per_call)
        # unrelated eager work on the same device between replays
        mixed.ix_gpu.search(mixed.q[:40].contiguous(), [0, 1, 17, 40], 5)
        torch.cuda.synchronize()
    # new query vectors in place (same offsets): the replay sees them
    q2, off2 = synth.make_fresh_queries(len(SIZES), 256, 384, 12, db_seed=5, seed=77, device="cpu", sizes=SIZES)
    assert np.array_equal(off2, mixed.q_off)
    q.copy_(q2.cuda())
    ref2 = [to_np(t) for t in mixed.ix_gpu.search(q, mixed.q_off, K)]
    _same([to_np(t) for t in b.run()], ref2)
    assert not np.array_equal(ref2[0], per_call[0])
    b.close()


def test_autotuner_picks_a_timed_shape_and_caches_it(mixed, per_call):
    from paper_2412_03301_amd import bvs
    _say("autotune")
    b = bvs.Batch(mixed.ix_gpu, mixed.q, mixed.q_off, K, graph=True)
    info = b.info()
    tried = info["tried"]
    if info["from_cache"]:
        assert not tried
    else:
        assert len(tried) >= 2 and all(ms > 0 for _, _, ms in tried)
        assert (0, 0) in [t[:2] for t in tried]   # the phase sequence is timed too
        best = min(tried, key=lambda t: t[2])
        assert (info["lds_rows"], info["waves"]) == best[:2]
    _same([to_np(t) for t in b.run()], per_call)
    b2 = bvs.Batch(mixed.ix_gpu, mixed.q, mixed.q_off, K, graph=False)
    i2 = b2.info()
    assert i2["from_cache"] and not i2["tried"]
    assert (i2["lds_rows"], i2["waves"]) == (info["lds_rows"], info["waves"])
    _same([to_np(t) for t in b2.run()], per_call)
    b.close()
    b2.close()


@pytest.mark.parametrize("env", [{"BVS_APPEND_CAP": "8"}, {"BVS_SELECT": "dense"}, {"BVS_APPEND_CAP": "300"}])
def test_batch_selection_paths(mixed, per_call, monkeypatch, env):
    """The dense fallback decided on the device, inside the graph."""
    from paper_2412_03301_amd import bvs
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    _say(f"selection {env}")
    b = bvs.Batch(mixed.ix_gpu, mixed.q, mixed.q_off, K, lds_rows=64, waves=4, graph=True)
    for _ in range(2):
        _same([to_np(t) for t in b.run()], per_call)
    b.close()


def test_screen_on_and_off_agree(mixed, per_call, monkeypatch):
    """The high-plane screen (a pass of its own in the per-call search, inside
    the persistent kernel in a batch) rejects candidates only when they
    provably cannot be among the k nearest: results with it switched off are
    identical, and with it on the per-call search does reject some.  (In a
    batch a later chunk screens only if its query's bound was published
    before the chunk started, which depends on timing; with 24 queries the
    chunks mostly start together.)"""
    from paper_2412_03301_amd import bvs
    _say("screen on/off")
    counts = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("BVS_SCREEN", flag)
        bvs.profile_enable(False, counters=True)
        _same([to_np(t) for t in mixed.ix_gpu.search(mixed.q, mixed.q_off, K)], per_call)
        counts[("call", flag)] = bvs.profile_counters()
        b = bvs.Batch(mixed.ix_gpu, mixed.q, mixed.q_off, K, lds_rows=64, waves=4, graph=False)
        bvs.profile_enable(False, counters=True)
        _same([to_np(t) for t in b.run()], per_call)
        counts[("batch", flag)] = bvs.profile_counters()
        bvs.profile_enable(False)
        b.close()
    on, off = counts[("call", "1")], counts[("call", "0")]
    assert on["rerank_screened"] > 0 and on["rerank_screen_vectors"] > 0
    for kind in ("call", "batch"):
        on, off = counts[(kind, "1")], counts[(kind, "0")]
        assert off["rerank_screened"] == 0 and off["rerank_screen_vectors"] == 0, kind
        assert on["rerank_screened"] <= on["rerank_abandoned"], kind
        assert on["rerank_candidates"] == off["rerank_candidates"], kind


def test_batch_single_query_and_k(mixed, oracle_res):
    from paper_2412_03301_amd import bvs
    i = SIZES.index(256)
    o0, o1 = mixed.q_off[i], mixed.q_off[i + 1]
    b = bvs.Batch(mixed.ix_gpu, mixed.q[o0:o1].contiguous(), [0, o1 - o0], 3, lds_rows=32, waves=2, graph=True)
    ids, dist, cnt = [to_np(t) for t in b.run()]
    r = oracle_res[i]
    assert cnt[0] == 3
    assert ids[0].view(np.uint32).astype(np.int64).tolist() == r["ids"][:3].tolist()
    b.close()


def test_batch_rejects_off_grid_queries(mixed):
    from paper_2412_03301_amd import bvs
    bad = mixed.q.clone()
    bad[5, 7] += 1e-4
    b = bvs.Batch(mixed.ix_gpu, bad, mixed.q_off, K, lds_rows=32, waves=4, graph=True)
    b.launch()
    with pytest.raises(bvs.BvsError) as e:
        b.status()
    assert e.value.status == bvs.BVS_ERANGE
    bad[5, 7] -= 1e-4
    b.launch()
    b.status()
    b.close()


def test_batch_tiny_subset_queries_match_oracle():
    from paper_2412_03301_amd import bvs
    _say("tiny subset queries, d=128")
    case = build_case(5000, 8, 32, 128, 50, 1024, 8, 32, 200, 16)
    res = [search.search(case.ix_oracle, case.query(i), A=3, M=1, T=200, k=10) for i in range(16)]
    b = bvs.Batch(case.ix_gpu, case.q, case.q_off, 10, graph=True)
    _check_oracle(res, *[to_np(t) for t in b.run()])
    b.close()


def test_batch_argument_errors(mixed):
    import ctypes as C
    from paper_2412_03301_amd import bvs
    L = bvs.lib()
    ix = mixed.ix_gpu
    off = np.asarray(mixed.q_off, np.uint64)

    def create(k=K, rows=0, waves=0, flags=0, offsets=off, n=len(SIZES)):
        cfg = bvs.BatchConfig(rows, waves, 1, flags)
        h = C.c_void_p()
        st = L.bvs_batch_create(ix._h, offsets.ctypes.data_as(bvs.PU64), n, k, C.byref(cfg), C.byref(h))
        return st, h

    assert create(k=0)[0] == bvs.BVS_EINVAL
    assert create(k=65)[0] == bvs.BVS_EINVAL
    assert create(rows=40)[0] == bvs.BVS_EINVAL
    assert create(rows=256)[0] == bvs.BVS_ENOTSUP     # 205 KB of LDS at d = 384
    assert create(waves=3)[0] == bvs.BVS_EINVAL
    assert create(flags=2)[0] == bvs.BVS_EINVAL
    assert create(rows=32, flags=bvs.BVS_BATCH_PHASES)[0] == bvs.BVS_EINVAL
    big = np.array([0, 257], np.uint64)
    assert create(offsets=big, n=1)[0] == bvs.BVS_ENOTSUP
    st, h = create(rows=32, waves=4)
    assert st == 0
    assert L.bvs_batch_launch(h, None) == bvs.BVS_ESTATE
    fake = C.c_void_p(mixed.q.data_ptr())
    assert L.bvs_batch_bind(h, fake, fake, 16, fake, fake, fake, None) == bvs.BVS_ENOSPC
    info = bvs.BatchInfo()
    assert L.bvs_batch_get_info(h, C.byref(info)) == 0
    ws = torch.empty(int(info.workspace_bytes), dtype=torch.uint8, device="cuda")
    out = torch.empty(len(SIZES) * K * 3, dtype=torch.int32, device="cuda")
    # graph capture on the null stream is refused
    st = L.bvs_batch_bind(h, C.c_void_p(mixed.q.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                          C.c_void_p(out.data_ptr()), C.c_void_p(out.data_ptr() + 4 * len(SIZES) * K),
                          C.c_void_p(out.data_ptr() + 8 * len(SIZES) * K), None)
    assert st == bvs.BVS_EINVAL
    L.bvs_batch_destroy(h)
