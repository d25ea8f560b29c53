"""Parity at full size: 1,000,000 sets (sizes 5-100, d = 384), L = 4096,
s = 16, wta_k = 64, T = 1000, and the whole batch of 1,024 queries in one
call, as the benchmark runs it.  The oracle cannot rebuild a million-set
index, so it checks sampled outputs one by one from the raw vectors:
query sketches, database sketches of sampled sets, the scores and order of
the returned candidates, that sampled sets left out of F2 rank after it,
exact distances of the returned results, and the same for brute force."""
import numpy as np
import pytest
import torch

from oracle import filter as flt
from oracle import flyhash, hausdorff, prng, sketch
from paper_2412_03301_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N_SETS, LO, HI, D, TOPICS = 1_000_000, 5, 100, 384, 10_000
L, S, K_WTA, T, K = 4096, 16, 64, 1000, 10
N_Q = 1024
CHECK_Q = (3, 255, 700, 1021)


@pytest.fixture(scope="module")
def big():
    from paper_2412_03301_amd import bvs
    print("[scale] generating 1M sets on the GPU", flush=True)
    dev = torch.device("cuda:0")
    db = synth.make_database(N_SETS, LO, HI, D, TOPICS, seed=0, device=dev)
    q, q_off, _ = synth.make_subset_queries(db, N_Q, seed=1)
    p = bvs.Params.make(dim=D, code_bits=L, fan_in=S, wta_k=K_WTA, access_lists=3, min_count=1, top_t=T, seed=0)
    print("[scale] building the index", flush=True)
    ix = bvs.Index(p, db.vectors, db.offsets)
    idx = prng.projection_rows(0, D, L, S)
    return dict(db=db, q=q.contiguous(), q_off=q_off, ix=ix, idx=idx)


def _set_vectors(big, j):
    o = big["db"].offsets
    return big["db"].vectors[o[j]:o[j + 1]].cpu().numpy().astype(np.float64)


def _query(big, i):
    return big["q"][big["q_off"][i]:big["q_off"][i + 1]].cpu().numpy().astype(np.float64)


def _oracle_sketch(big, j):
    H = flyhash.codes(_set_vectors(big, j), big["idx"], K_WTA)
    off = np.array([0, len(H)])
    return sketch.count_bloom(H, off)[0], sketch.binary_bloom(H, off)[0]


def test_query_sketches_at_scale(big):
    cq, sq, pos = big["ix"].query_sketch(big["q"], big["q_off"])
    cq, sq, pos = cq.cpu().numpy().view(np.uint16), sq.cpu().numpy().view(np.uint64), pos.cpu().numpy()
    for i in CHECK_Q:
        C_Q, S_Q = flt.query_sketches(flyhash.codes(_query(big, i), big["idx"], K_WTA))
        assert np.array_equal(cq[i].astype(np.int64), C_Q)
        assert np.array_equal(sq[i], flyhash.pack(S_Q[None])[0])
        assert pos[i].tolist() == flt.top_positions(C_Q, 3).tolist()


def test_database_sketches_sampled(big):
    cnt, bits = big["ix"].sketch_views()
    rng = np.random.default_rng(0)
    sets = rng.choice(N_SETS, 40, replace=False).tolist() + [0, N_SETS - 1]
    for j in sets:
        C, B = _oracle_sketch(big, j)
        assert np.array_equal(cnt[:, j].cpu().numpy().astype(np.int64), C)
        w = bits[:, j, :].cpu().numpy().view(np.uint64).reshape(-1)
        assert np.array_equal(w, flyhash.pack(B[None])[0])


def test_candidates_and_results_sampled(big):
    ix = big["ix"]
    f2, f2s, f2c = ix.candidates(big["q"], big["q_off"])
    f2, f2s, f2c = f2.cpu().numpy().view(np.uint32), f2s.cpu().numpy().view(np.uint16), f2c.cpu().numpy()
    ids, dist, cnt = ix.search(big["q"], big["q_off"], K)
    ids, dist, cnt = ids.cpu().numpy().view(np.uint32), dist.cpu().numpy(), cnt.cpu().numpy()
    rng = np.random.default_rng(1)
    for i in CHECK_Q:
        Q = _query(big, i)
        C_Q, S_Q = flt.query_sketches(flyhash.codes(Q, big["idx"], K_WTA))
        P = flt.top_positions(C_Q, 3)
        assert f2c[i] == T
        keys = list(zip(f2s[i].astype(int).tolist(), f2[i].astype(int).tolist()))
        assert keys == sorted(keys)
        # scores and membership of sampled candidates, from the raw vectors
        for t in sorted(rng.choice(T, 60, replace=False).tolist()) + [T - 1]:
            C, B = _oracle_sketch(big, int(f2[i, t]))
            assert flt.first_filter(C[None], P, 1)[0]
            assert flt.hamming(S_Q, B[None])[0] == f2s[i, t]
        # sampled sets outside F2 are non-members or rank after the last candidate
        last = keys[-1]
        inside = set(f2[i].tolist())
        for j in rng.choice(N_SETS, 150, replace=False).tolist():
            if j in inside:
                continue
            C, B = _oracle_sketch(big, j)
            if flt.first_filter(C[None], P, 1)[0]:
                assert (int(flt.hamming(S_Q, B[None])[0]), j) > last
        # results: the first K of the candidate list by (exact Hausdorff^2,
        # id), the oracle's exact value computed for every one of the T
        # candidates (this is where the screen and the bound phases discard
        # most of them), with exact distances
        assert cnt[i] == K
        h2_all = np.array([hausdorff.hausdorff_sq(Q, _set_vectors(big, int(j))) for j in f2[i]])
        order = np.lexsort((f2[i].astype(np.int64), h2_all))[:K]
        assert ids[i].astype(np.int64).tolist() == f2[i][order].astype(np.int64).tolist()
        np.testing.assert_allclose(dist[i], np.sqrt(h2_all[order]), rtol=1e-5, atol=0)


def test_bruteforce_sampled(big):
    ix = big["ix"]
    nb = 8
    qb = big["q"][: int(big["q_off"][nb])].contiguous()
    ids, dist, cnt = ix.bruteforce(qb, big["q_off"][: nb + 1], K)
    ids, dist = ids.cpu().numpy().view(np.uint32), dist.cpu().numpy()
    rng = np.random.default_rng(2)
    for i in (0, 5):
        Q = _query(big, i)
        h2 = [hausdorff.hausdorff_sq(Q, _set_vectors(big, int(j))) for j in ids[i]]
        np.testing.assert_allclose(dist[i], np.sqrt(h2), rtol=1e-5, atol=0)
        res = list(zip(h2, ids[i].astype(int).tolist()))
        assert res == sorted(res)
        chosen = set(ids[i].tolist())
        for j in rng.choice(N_SETS, 400, replace=False).tolist():
            if j not in chosen:
                assert (hausdorff.hausdorff_sq(Q, _set_vectors(big, j)), j) > res[-1]


def test_screen_identity_whole_batch(big, monkeypatch):
    """Every one of the 1,024 queries gets the same results with the
    high-plane screen on and off."""
    from paper_2412_03301_amd import bvs
    out = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("BVS_SCREEN", flag)
        bvs.profile_enable(False, counters=True)
        out[flag] = [t.cpu().numpy() for t in big["ix"].search(big["q"], big["q_off"], K)]
        out[flag + "c"] = bvs.profile_counters()
        bvs.profile_enable(False)
    assert out["1c"]["rerank_screened"] > 0 and out["0c"]["rerank_screened"] == 0
    for a, b in zip(out["1"], out["0"]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape", ["phases", "persistent"])
def test_batched_plan_identity_whole_batch(big, shape):
    """The batched plan, replayed from its graph, returns for every one of the
    1,024 queries exactly what one search call over the batch returns, with
    the re-rank as the phase sequence by size class and as the persistent
    launch."""
    from paper_2412_03301_amd import bvs
    print(f"[scale] batched plan ({shape}) against one search call", flush=True)
    ref = [t.cpu().numpy() for t in big["ix"].search(big["q"], big["q_off"], K)]
    kw = dict(phases=True) if shape == "phases" else dict(lds_rows=64, waves=4)
    b = bvs.Batch(big["ix"], big["q"], big["q_off"], K, graph=True, **kw)
    for _ in range(2):   # two replays
        got = [t.cpu().numpy() for t in b.run()]
        for a, c in zip(got, ref):
            assert np.array_equal(a, c)
    b.close()
