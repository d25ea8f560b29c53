"""Precision form of the re-rank on the GPU against the oracle: the BF16 and
FP8 E4M3 approximate Hausdorff values (within float32 accumulation of the
oracle's float64 evaluation of the same quantised values), the re-check
selection, and the final results (exact ids and distances)."""
import numpy as np
import pytest
import torch

from oracle import lowp, search
from tests.gpu_util import build_case, to_np

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5
APPROX_ABS, APPROX_REL = 2e-5, 1e-5
FMTS = ("bf16", "fp8")


def _say(msg):
    print(f"[lowp] {msg}", flush=True)


CASES = {
    # name: (n_sets, lo, hi, d, topics, L, s, wta_k, T, n_q, queries)
    "d128": (3000, 5, 40, 128, 30, 1024, 8, 32, 200, 8, "subset"),
    "d768": (1200, 5, 60, 768, 12, 2048, 8, 32, 150, 6, "subset"),
    "d768_big_queries": (800, 5, 60, 768, 8, 2048, 8, 32, 100, 4, [81, 130, 256, 17]),
    "d100_pad": (900, 2, 30, 100, 10, 512, 4, 16, 120, 5, "subset"),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    n, lo, hi, d, top, L, s, k, T, nq, qk = CASES[request.param]
    _say(f"case {request.param}")
    c = build_case(n, lo, hi, d, top, L, s, k, T, nq, seed=9, queries=qk)
    for f in FMTS:
        c.ix_gpu.attach_lowp(f)
    return c, T


@pytest.mark.parametrize("fmt", FMTS)
def test_approx_values_match_oracle(case, fmt):
    c, T = case
    ids, _, cnt = c.ix_gpu.candidates(c.q, c.q_off)
    m = 64
    sel = ids[:, :m].contiguous()
    got = to_np(c.ix_gpu.hausdorff_lowp(c.q, c.q_off, sel, fmt)).astype(np.float64)
    sel = to_np(sel).view(np.uint32)
    cnt = to_np(cnt)
    for i in range(len(c.q_off) - 1):
        Q = c.query(i)
        for t in range(min(m, int(cnt[i]))):
            j = int(sel[i, t])
            ref = lowp.approx_hausdorff_sq(Q, c.ix_oracle.members(j), fmt)
            assert abs(got[i, t] - ref) <= APPROX_ABS + APPROX_REL * ref, (i, t, j, got[i, t], ref)


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("margin", [0.0, 0.02, 0.1])
def test_search_lowp_matches_oracle(case, fmt, margin):
    c, T = case
    k = 10
    ids, dist, cnt, rech = [to_np(t) for t in c.ix_gpu.search_lowp(c.q, c.q_off, k, fmt, margin)]
    ids = ids.view(np.uint32)
    for i in range(len(c.q_off) - 1):
        r = lowp.search_lowp(c.ix_oracle, c.query(i), A=3, M=1, T=T, k=k, fmt=fmt, margin=margin)
        n = len(r["ids"])
        assert cnt[i] == n
        # re-checked count: equal up to candidates whose value sits at the threshold
        ah = np.sort(r["approx_h2"])
        if len(ah) >= k:
            thr = float(lowp.recheck_threshold(ah[k - 1], margin))
            near = np.sum(np.abs(ah - thr) <= APPROX_ABS + APPROX_REL * thr + 1e-6 * thr)
            near += np.sum(np.abs(ah - ah[k - 1]) <= APPROX_ABS + APPROX_REL * ah[k - 1])
            assert abs(int(rech[i]) - len(r["recheck"])) <= near
            assert rech[i] >= k
        else:
            assert rech[i] == len(ah)
        if int(rech[i]) == len(r["recheck"]):
            assert ids[i, :n].astype(np.int64).tolist() == r["ids"].tolist()
            np.testing.assert_allclose(dist[i, :n], np.sqrt(r["h2"]), rtol=REL_TOL, atol=0)
        else:
            # different boundary sets: the results are still exact distances, sorted
            h2 = [float(np.float64(search.hausdorff_sq(c.query(i), c.ix_oracle.members(int(j))))) for j in ids[i, :n]]
            np.testing.assert_allclose(dist[i, :n], np.sqrt(h2), rtol=REL_TOL, atol=0)


@pytest.mark.parametrize("fmt", FMTS)
def test_large_margin_equals_exact_search(case, fmt):
    c, T = case
    a = [to_np(t) for t in c.ix_gpu.search(c.q, c.q_off, 10)]
    b = [to_np(t) for t in c.ix_gpu.search_lowp(c.q, c.q_off, 10, fmt, margin=1e6)]
    for x, y in zip(a, b[:3]):
        assert np.array_equal(x, y)
    _, _, f2c = c.ix_gpu.candidates(c.q, c.q_off)
    assert np.array_equal(b[3], to_np(f2c))


def test_lowp_argument_errors():
    from paper_2412_03301_amd import bvs
    c = build_case(300, 2, 10, 64, 4, 256, 4, 8, 40, 3, seed=2)
    with pytest.raises(bvs.BvsError) as e:
        c.ix_gpu.search_lowp(c.q, c.q_off, 5, "bf16")
    assert e.value.status == bvs.BVS_ESTATE
    c.ix_gpu.attach_lowp("fp8")
    with pytest.raises(bvs.BvsError) as e:
        c.ix_gpu.search_lowp(c.q, c.q_off, 5, "fp8", margin=-0.5)
    assert e.value.status == bvs.BVS_EINVAL
    with pytest.raises(bvs.BvsError) as e:
        c.ix_gpu.search_lowp(c.q, c.q_off, 5, "fp8", margin=float("nan"))
    assert e.value.status == bvs.BVS_EINVAL
    import ctypes as C
    out = C.c_uint64()
    assert bvs.lib().bvs_lowp_bytes(c.ix_gpu._h, 3, C.byref(out)) == bvs.BVS_EINVAL
    ids, dist, cnt, rech = c.ix_gpu.search_lowp(c.q, c.q_off, 5, "fp8")
    assert (to_np(cnt) == 5).all()
