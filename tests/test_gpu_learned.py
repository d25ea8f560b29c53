"""Learned projection on the GPU against the oracle: codes of the bfloat16
network (identical but for values within float32-accumulation distance of
the winner-take-all boundary), the whole search on a learned index, the
batched and precision forms on it, the training gradients (against the
float64 chain rule) and a loss that decreases."""
import numpy as np
import pytest
import torch

from oracle import learned, search
from paper_2412_03301_amd import synth
from tests.gpu_util import to_np

pytestmark = pytest.mark.gpu

D, H, L, K = 64, 96, 512, 16
REL_TOL = 1e-5


def _say(msg):
    print(f"[learned] {msg}", flush=True)


@pytest.fixture(scope="module")
def case():
    from paper_2412_03301_amd import bvs
    _say("building learned index d=64 H=96 L=512")
    db = synth.make_database(1500, 3, 20, D, 10, seed=7)
    q, q_off, _ = synth.make_subset_queries(db, 8, seed=8)
    w = bvs.mlp_weights(D, H, L, seed=11)
    p = bvs.Params.make(dim=D, code_bits=L, fan_in=4, wta_k=K, top_t=100, seed=0)
    ix = bvs.Index(p, db.vectors.cuda(), db.offsets, mlp=(H, w))
    W = [t.cpu().numpy().astype(np.float64) for t in bvs.unpack_mlp(w, D, H, L)]
    X = db.vectors.numpy().astype(np.float64)
    _, _, y = learned.mlp(X, *W, quantised=True)
    yq = learned.bf16(y)
    Hc = learned.wta_codes(yq, K)
    ix_o = search.index_from_codes(X, db.offsets, Hc, K)
    return dict(db=db, q=q.cuda().contiguous(), q_np=q.numpy().astype(np.float64), q_off=q_off, w=w, W=W, ix=ix,
                ix_o=ix_o, yq=yq, Hc=Hc, X=X)


def _codes_close(got_words, yq, Hc):
    """Codes equal the oracle's except where the oracle's values tie with the
    k-th within two bfloat16 ulps."""
    got = np.unpackbits(got_words.view(np.uint8), axis=1, bitorder="little").astype(bool)
    diff = np.flatnonzero((got != Hc).any(axis=1))
    for i in diff:
        kth = np.sort(yq[i])[::-1][K - 1]
        ulp = 2.0 ** (np.floor(np.log2(abs(kth) + 1e-30)) - 7)
        pos = np.flatnonzero(got[i] != Hc[i])
        assert np.all(np.abs(yq[i, pos] - kth) <= 2 * ulp), (i, yq[i, pos], kth)
    return len(diff) / len(Hc)


def test_learned_codes_match_oracle(case):
    codes = to_np(case["ix"].encode(case["db"].vectors.cuda())).view(np.uint64)
    frac = _codes_close(codes, case["yq"], case["Hc"])
    assert frac <= 0.01
    assert (np.unpackbits(codes.view(np.uint8), axis=1).sum(axis=1) == K).all()


def test_learned_search_matches_oracle(case):
    ids, dist, cnt = [to_np(t) for t in case["ix"].search(case["q"], case["q_off"], 10)]
    ids = ids.view(np.uint32)
    W = case["W"]
    for i in range(len(case["q_off"]) - 1):
        Q = case["q_np"][case["q_off"][i]:case["q_off"][i + 1]]
        HQ = learned.wta_codes(learned.bf16(learned.mlp(Q, *W, quantised=True)[2]), K)
        r = search.search_codes(case["ix_o"], Q, HQ, A=3, M=1, T=100, k=10)
        assert cnt[i] == len(r["ids"])
        assert ids[i, :cnt[i]].astype(np.int64).tolist() == r["ids"].tolist()
        np.testing.assert_allclose(dist[i, :cnt[i]], np.sqrt(r["h2"]), rtol=REL_TOL, atol=0)


def test_learned_index_in_batched_and_precision_forms(case):
    from paper_2412_03301_amd import bvs
    ref = [to_np(t) for t in case["ix"].search(case["q"], case["q_off"], 10)]
    b = bvs.Batch(case["ix"], case["q"], case["q_off"], 10, lds_rows=32, waves=4, graph=True)
    out = [to_np(t) for t in b.run()]
    for x, y in zip(out, ref):
        assert np.array_equal(x, y)
    b.close()
    case["ix"].attach_lowp("fp8")
    lp = [to_np(t) for t in case["ix"].search_lowp(case["q"], case["q_off"], 10, "fp8", margin=1e6)]
    for x, y in zip(lp[:3], ref):
        assert np.array_equal(x, y)


def _train_case(seed=5):
    rng = np.random.default_rng(seed)
    db = synth.make_database(40, 2, 9, D, 4, seed=seed)
    trip = np.array([[i, (i + 1) % 40, (i + 17) % 40] for i in range(40)], np.uint32)
    rng.shuffle(trip)
    return db, trip


def test_training_gradients_match_oracle():
    from paper_2412_03301_amd import bvs
    db, trip = _train_case()
    w = bvs.mlp_weights(D, H, L, seed=3)
    cfg = bvs.TrainConfig(D, H, L, K, 64, 1, 1e-3, 0.5, 4.0, 0, 0)
    tr = bvs.Trainer(cfg, db.vectors.cuda(), db.offsets, max_batch_rows=64 * 3 * 9)
    loss, g = tr.gradients(w, trip)
    W = [t.cpu().numpy().astype(np.float64) for t in bvs.unpack_mlp(w, D, H, L)]
    sets = [db.vectors[db.offsets[j]:db.offsets[j + 1]].numpy().astype(np.float64) for j in range(40)]
    ref_loss, ref = learned.triplet_grads(W, sets, [tuple(int(x) for x in t) for t in trip], K, 0.5, 4.0)
    assert ref_loss > 0
    assert abs(loss - ref_loss) <= 0.02 * ref_loss
    got = [t.cpu().numpy().astype(np.float64) for t in bvs.unpack_mlp(g, D, H, L)]
    for a, r in zip(got, ref):
        cos = float((a * r).sum() / (np.linalg.norm(a) * np.linalg.norm(r) + 1e-30))
        assert cos >= 0.98, cos
        assert abs(np.linalg.norm(a) - np.linalg.norm(r)) <= 0.05 * np.linalg.norm(r)


def test_training_lowers_the_loss():
    from paper_2412_03301_amd import bvs
    db, trip = _train_case(6)
    w = bvs.mlp_weights(D, H, L, seed=4)
    cfg = bvs.TrainConfig(D, H, L, K, 16, 6, 3e-3, 0.5, 4.0, 0, 9)
    tr = bvs.Trainer(cfg, db.vectors.cuda(), db.offsets, max_batch_rows=16 * 3 * 9)
    losses = tr.train(w, trip)
    assert len(losses) == 6 and all(np.isfinite(losses))
    assert losses[-1] < 0.8 * losses[0], losses


def test_training_resumes_from_a_checkpoint():
    # four epochs in one call against two calls of two epochs with the
    # weights and the optimizer state copied to the host and back between
    # them: the same batches and Adam steps, equal up to the order of the
    # gradients' floating-point sums
    from paper_2412_03301_amd import bvs
    db, trip = _train_case(6)
    w0 = bvs.mlp_weights(D, H, L, seed=5)
    tr4 = bvs.Trainer(bvs.TrainConfig(D, H, L, K, 16, 4, 3e-3, 0.5, 4.0, 0, 9), db.vectors.cuda(), db.offsets,
                      max_batch_rows=16 * 3 * 9)
    tr2 = bvs.Trainer(bvs.TrainConfig(D, H, L, K, 16, 2, 3e-3, 0.5, 4.0, 0, 9), db.vectors.cuda(), db.offsets,
                      max_batch_rows=16 * 3 * 9)
    w_one = w0.clone()
    losses_one = tr4.train(w_one, trip)
    w_res = w0.clone()
    st = tr2.new_state()
    l1 = tr2.train_resume(w_res, trip, st)
    ckpt_w, ckpt_s = w_res.cpu().clone(), st.cpu().clone()
    del w_res, st
    w_res, st = ckpt_w.cuda(), ckpt_s.cuda()
    l2 = tr2.train_resume(w_res, trip, st)
    np.testing.assert_allclose(l1 + l2, losses_one, rtol=2e-3)
    a, b = w_res.cpu().numpy().astype(np.float64), w_one.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b)
    # the header counts the Adam steps and epochs done
    n_batches = -(-len(trip) // 16)
    hdr = st.cpu().numpy()[-256:].view(np.uint64)[:2]
    assert hdr.tolist() == [4 * n_batches, 4]
