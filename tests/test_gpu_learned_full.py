"""The learned projection at the precision-form shapes (d = 768, hidden
1024, L = 4096, winner-take-all 64): the kernels instantiated there
(k_wta_rows<64>, the 64-word training kernels, the 768 -> 1024 -> 4096 GEMM
tiles) against the oracle.

Exact-forward inputs: rows with +-1/4 on 24 coordinates and weights that are
multiples of 1/16 in [-1/2, 1/2], so x, W1, relu(W1 x + b1) and W2 are
bfloat16 values and every forward sum is exact in float32 in any order; the
GPU and the oracle then hold the same outputs y, and the codes must agree bit
for bit (ties, which are many, to the lower index).  Gradients are compared
element by element with the oracle's bfloat16-operand chain rule, within a
tolerance derived from where they can still differ: one bfloat16 rounding
(of dy or dpre) that lands on the other side of a rounding boundary, at most
one ulp = 2^-7 of the rounded value, and float32 arithmetic in the soft
forms and sums, each bounded by the sum of absolute terms."""
import numpy as np
import pytest
import torch

from oracle import learned, search
from paper_2412_03301_amd import synth
from tests.gpu_util import to_np

pytestmark = pytest.mark.gpu

D, H, L, K = 768, 1024, 4096, 64
REL_TOL = 1e-5


def _say(msg):
    print(f"[learned-768] {msg}", flush=True)


def _exact_weights(rng):
    W = [rng.integers(-8, 9, (H, D)) / 16.0, rng.integers(-4, 5, H) / 16.0,
         rng.integers(-8, 9, (L, H)) / 16.0, rng.integers(-4, 5, L) / 16.0]
    packed = torch.from_numpy(np.concatenate([w.reshape(-1) for w in W]).astype(np.float32))
    return W, packed


def _exact_rows(rng, n, nnz=24):
    X = np.zeros((n, D), np.float32)
    for r in range(n):
        X[r, rng.choice(D, nnz, replace=False)] = rng.choice([-0.25, 0.25], nnz)
    return X


def _exact_sets(rng, sizes):
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return _exact_rows(rng, int(off[-1])), off


@pytest.fixture(scope="module")
def full():
    from paper_2412_03301_amd import bvs
    _say("exact-forward learned index: 200 sets of 5-100 vectors, d=768, H=1024, L=4096, k=64")
    rng = np.random.default_rng(21)
    W, packed = _exact_weights(rng)
    X, off = _exact_sets(rng, rng.integers(5, 101, 200))
    p = bvs.Params.make(dim=D, code_bits=L, fan_in=16, wta_k=K, top_t=150, seed=0)
    ix = bvs.Index(p, torch.from_numpy(X).cuda(), off, mlp=(H, packed.cuda()))
    X64 = X.astype(np.float64)
    _, _, y = learned.mlp(X64, *W, quantised=True)
    Hc = learned.wta_codes(learned.bf16(y), K)
    # queries: 6 database sets with every third member dropped
    qs = [X[off[j]:off[j + 1]][np.arange(off[j + 1] - off[j]) % 3 != 2] for j in (3, 50, 77, 120, 160, 199)]
    q_off = np.concatenate([[0], np.cumsum([len(x) for x in qs])]).astype(np.int64)
    Q = np.concatenate(qs)
    return dict(ix=ix, W=W, X=X, off=off, Hc=Hc, y=y, q=torch.from_numpy(Q).cuda().contiguous(),
                q_np=Q.astype(np.float64), q_off=q_off)


def test_exact_forward_precondition(full):
    # sums of absolute products, in units of the operands' common quantum,
    # stay below 2^24: float32 holds every partial sum exactly
    X, (W1, b1, W2, b2) = full["X"].astype(np.float64), full["W"]
    pre_abs = np.abs(X) @ np.abs(W1).T + np.abs(b1)
    assert pre_abs.max() * 2 ** 6 < 2 ** 24
    h = np.maximum(X @ W1.T + b1, 0)
    assert np.array_equal(learned.bf16(h), h)
    y_abs = h @ np.abs(W2).T + np.abs(b2)
    assert y_abs.max() * 2 ** 10 < 2 ** 24


def test_codes_bit_exact_at_full_shape(full):
    codes = to_np(full["ix"].encode(torch.from_numpy(full["X"]).cuda())).view(np.uint64)
    got = np.unpackbits(codes.view(np.uint8), axis=1, bitorder="little").astype(bool)
    assert got.shape == full["Hc"].shape
    assert np.array_equal(got, full["Hc"])
    # ties at the winner-take-all boundary are common with these weights
    yq = learned.bf16(full["y"])
    kth = -np.sort(-yq, axis=1)[:, K - 1]
    assert ((yq == kth[:, None]).sum(axis=1) > 1).mean() > 0.1


def test_search_at_full_shape(full):
    ix_o = search.index_from_codes(full["X"].astype(np.float64), full["off"], full["Hc"], K)
    ids, dist, cnt = [to_np(t) for t in full["ix"].search(full["q"], full["q_off"], 10)]
    ids = ids.view(np.uint32)
    W = full["W"]
    for i in range(len(full["q_off"]) - 1):
        Q = full["q_np"][full["q_off"][i]:full["q_off"][i + 1]]
        HQ = learned.wta_codes(learned.bf16(learned.mlp(Q, *W, quantised=True)[2]), K)
        r = search.search_codes(ix_o, Q, HQ, A=3, M=1, T=150, k=10)
        assert cnt[i] == len(r["ids"])
        assert ids[i, :cnt[i]].astype(np.int64).tolist() == r["ids"].tolist()
        np.testing.assert_allclose(dist[i, :cnt[i]], np.sqrt(r["h2"]), rtol=REL_TOL, atol=0)


def test_gradients_elementwise_at_full_shape():
    from paper_2412_03301_amd import bvs
    _say("training gradients at d=768, H=1024, L=4096 (16 triplets of distinct sets)")
    rng = np.random.default_rng(22)
    W, packed = _exact_weights(rng)
    X, off = _exact_sets(rng, rng.integers(5, 41, 48))
    trip = np.arange(48, dtype=np.uint32).reshape(16, 3)       # every set in one triplet
    tau, margin = 0.5, 16384.0                                  # every hinge active
    cfg = bvs.TrainConfig(D, H, L, K, 16, 1, 1e-3, tau, margin, 0, 0)
    tr = bvs.Trainer(cfg, torch.from_numpy(X).cuda(), off, max_batch_rows=int(off[-1]))
    loss, g = tr.gradients(packed.cuda(), trip)
    got = [t.cpu().numpy().astype(np.float64) for t in bvs.unpack_mlp(g, D, H, L)]
    sets = [X[off[j]:off[j + 1]].astype(np.float64) for j in range(48)]
    trace = []
    ref_loss, ref = learned.triplet_grads(W, sets, [tuple(int(x) for x in t) for t in trip], K, tau, margin,
                                          quantised=True, trace=trace)
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    # absolute-term bound of dS (each set is in exactly one triplet)
    nt = len(trip)
    S = [t[10] for t in trace]
    dS_abs = [None] * 48
    for q, p, n in trip.tolist():
        dS_abs[q] = 2.0 * (S[n] + S[p]) / nt
        dS_abs[p] = (1.0 + 2.0 * S[q]) / nt
        dS_abs[n] = (1.0 + 2.0 * S[q]) / nt
    aW2 = np.zeros((L, H))
    ab2 = np.zeros(L)
    aW1 = np.zeros((H, D))
    ab1 = np.zeros(H)
    for s, (x, pre, h, dy, dyq, dpre, dpreq, W2q, c, others, _) in enumerate(trace):
        dy_abs = dS_abs[s][None, :] * others * c * (1.0 - c) / tau      # >= |dy|
        B = dy_abs @ np.abs(W2q)                                          # >= |dh|
        aW2 += dy_abs.T @ np.abs(h)
        ab2 += dy_abs.sum(axis=0)
        A1 = (np.abs(dpre) + B) * (pre > 0)
        aW1 += A1.T @ np.abs(x)
        ab1 += A1.sum(axis=0)
    tol = 2.0 ** -6      # one bfloat16 ulp (2^-7) plus float32 terms, with room
    names = ("W1", "b1", "W2", "b2")
    for name, a, r, bound in zip(names, got, ref, (aW1, ab1, aW2, ab2)):
        err = np.abs(a - r)
        lim = tol * bound + 1e-12
        bad = np.argwhere(err > lim)
        assert len(bad) == 0, (name, len(bad), err.max(), a.reshape(-1)[:4], r.reshape(-1)[:4])
        # The bound above is the worst case; for W1 and b1 it is loose (dh sums
        # 4096 terms of both signs).  A flip of one rounding needs the two
        # sides' dy (float32 against float64 transcendentals, ~1e-6 apart) to
        # straddle a bfloat16 boundary, about one element in 4000, so the
        # total error stays near 1e-4 of the total gradient.
        agg = err.sum() / np.abs(r).sum()
        _say(f"{name}: max err {err.max():.3g}, total err / total |g| {agg:.3g}")
        assert agg <= 1e-3, (name, agg)


def test_realistic_codes_at_full_shape():
    """Grid vectors from the workload generator and the initialised network:
    float32 accumulation may split values the oracle (float64) sees equal,
    so codes agree except where the oracle's values tie with the k-th within
    two bfloat16 ulps, on at most 1 % of the vectors."""
    from paper_2412_03301_amd import bvs
    db = synth.make_database(60, 5, 100, D, 6, seed=9)
    w = bvs.mlp_weights(D, H, L, seed=12)
    p = bvs.Params.make(dim=D, code_bits=L, fan_in=16, wta_k=K, top_t=40, seed=0)
    ix = bvs.Index(p, db.vectors.cuda(), db.offsets, mlp=(H, w))
    Wn = [t.cpu().numpy().astype(np.float64) for t in bvs.unpack_mlp(w, D, H, L)]
    _, _, y = learned.mlp(db.vectors.numpy().astype(np.float64), *Wn, quantised=True)
    yq = learned.bf16(y)
    Hc = learned.wta_codes(yq, K)
    codes = to_np(ix.encode(db.vectors.cuda())).view(np.uint64)
    got = np.unpackbits(codes.view(np.uint8), axis=1, bitorder="little").astype(bool)
    assert (got.sum(axis=1) == K).all()
    diff = np.flatnonzero((got != Hc).any(axis=1))
    for i in diff:
        kth = np.sort(yq[i])[::-1][K - 1]
        ulp = 2.0 ** (np.floor(np.log2(abs(kth) + 1e-30)) - 7)
        pos = np.flatnonzero(got[i] != Hc[i])
        assert np.all(np.abs(yq[i, pos] - kth) <= 2 * ulp)
    assert len(diff) <= 0.01 * len(Hc)
