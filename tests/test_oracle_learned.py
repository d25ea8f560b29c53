"""Pins of the learned-projection oracle: it reduces to the random FlyHash
when the network is a fixed sparse projection, its soft sketches and soft
Hamming distance reduce to Defs. 10 and 11 on binary codes, and its
gradients match finite differences."""
import numpy as np

from oracle import filter as flt
from oracle import flyhash, learned, sketch
from oracle.prng import projection_matrix, projection_rows


def test_network_reduces_to_random_flyhash():
    rng = np.random.default_rng(0)
    d, L, s, k = 16, 128, 4, 8
    X = np.round(rng.normal(size=(30, d)) / 4 * 4096) / 4096
    idx = projection_rows(3, d, L, s)
    W2 = projection_matrix(idx, d)
    off = 10.0                              # keeps every hidden unit active
    W1, b1 = np.eye(d), np.full(d, off)
    b2 = -W2 @ b1
    _, _, y = learned.mlp(X, W1, b1, W2, b2)
    ref = flyhash.codes(X, idx, k)
    assert np.array_equal(learned.wta_codes(y, k), ref)


def test_wta_ties_and_thresholds():
    Y = np.zeros((2, 10))
    Y[1, [3, 7]] = 1.0
    c = learned.wta_codes(Y, 3)
    assert c[0].tolist() == [True] * 3 + [False] * 7
    assert np.flatnonzero(c[1]).tolist() == [0, 3, 7]
    assert learned.thresholds(np.array([[5.0, 1.0, 3.0, 2.0]]), 2).tolist() == [2.5]


def test_soft_forms_reduce_to_bloom_and_hamming_on_binary_codes():
    rng = np.random.default_rng(1)
    H = rng.random((12, 64)) < 0.2
    off = np.array([0, 5, 12])
    B = sketch.binary_bloom(H, off)
    for i in range(2):
        assert np.array_equal(learned.soft_sketch(H[off[i]:off[i + 1]].astype(float)), B[i].astype(float))
    assert learned.soft_hamming(B[0].astype(float), B[1].astype(float)) == flt.hamming(B[0], B[1:2])[0]


def test_soft_codes_approach_hard_codes():
    rng = np.random.default_rng(2)
    Y = rng.normal(size=(5, 40))
    c = learned.soft_codes(Y, 6, 1e-4)
    assert np.array_equal(c > 0.5, learned.wta_codes(Y, 6))


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    d, H, L, k = 6, 5, 12, 3
    W = [rng.normal(size=(H, d)) * 0.7, rng.normal(size=H) * 0.3, rng.normal(size=(L, H)) * 0.7,
         rng.normal(size=L) * 0.3]
    sets = [rng.normal(size=(m, d)) for m in (3, 2, 4, 1)]
    trip = [(0, 1, 2), (3, 2, 1), (1, 0, 3)]
    tau, margin = 0.5, 2.0
    t0 = learned.set_thresholds(W, sets, k)
    loss, grads = learned.triplet_grads(W, sets, trip, k, tau, margin)
    assert abs(loss - learned.triplet_loss(W, sets, trip, k, tau, margin, t0)) < 1e-12
    assert loss > 0
    eps = 1e-6
    for wi in range(4):
        flat = W[wi].reshape(-1)
        g = grads[wi].reshape(-1)
        for e in rng.choice(flat.size, min(6, flat.size), replace=False):
            old = flat[e]
            flat[e] = old + eps
            lp = learned.triplet_loss(W, sets, trip, k, tau, margin, t0)
            flat[e] = old - eps
            lm = learned.triplet_loss(W, sets, trip, k, tau, margin, t0)
            flat[e] = old
            num = (lp - lm) / (2 * eps)
            assert abs(num - g[e]) <= 1e-6 + 1e-5 * abs(num), (wi, e, num, g[e])


def _exact_forward_case(rng, d, H, L, sizes, nnz):
    """Inputs with entries in {0, +-1/4} (nnz per row) and weights that are
    multiples of 1/16 in [-1/2, 1/2]: every product operand is a bfloat16
    value and every forward sum is exact in float32 in any order."""
    W = [rng.integers(-8, 9, (H, d)) / 16.0, rng.integers(-4, 5, H) / 16.0,
         rng.integers(-8, 9, (L, H)) / 16.0, rng.integers(-4, 5, L) / 16.0]
    sets = []
    for m in sizes:
        X = np.zeros((m, d))
        for r in range(m):
            X[r, rng.choice(d, nnz, replace=False)] = rng.choice([-0.25, 0.25], nnz)
        sets.append(X)
    return W, sets


def test_quantised_gradients_within_rounding_of_float64_chain_rule():
    # On bfloat16-exact operands the quantised mode differs from the plain
    # chain rule (pinned by finite differences above) only by the bfloat16
    # rounding of dy and dpre before their products: at most one half-ulp,
    # 2^-8 of each rounded term, propagated through the sums of absolute
    # products.  A dropped rounding, a transposed operand or a wrong mask
    # would break either the bound or the equality below.
    rng = np.random.default_rng(4)
    d, H, L, k = 24, 16, 64, 8
    W, sets = _exact_forward_case(rng, d, H, L, (3, 5, 2, 4, 1), 6)
    trip = [(0, 1, 2), (3, 2, 4), (1, 0, 3), (4, 3, 0)]
    tau, margin = 0.5, 6.0
    trace = []
    lq, gq = learned.triplet_grads(W, sets, trip, k, tau, margin, quantised=True, trace=trace)
    lf, gf = learned.triplet_grads(W, sets, trip, k, tau, margin)
    assert lq == lf and lq > 0                  # the forward pass is exact: same loss
    u = 2.0 ** -8
    aW2 = sum(np.abs(t[3]).T @ np.abs(t[2]) for t in trace)
    # dpre differs by its own rounding (u |dpre|) and by dh's share of the
    # rounding of dy (u |dy| |W2|)
    aW1 = sum((np.abs(t[5]) + np.abs(t[3]) @ np.abs(t[7])).T @ np.abs(t[0]) for t in trace)
    ab1 = sum((u * (np.abs(t[3]) @ np.abs(t[7]))).sum(axis=0) for t in trace)
    assert np.all(np.abs(gq[2] - gf[2]) <= u * aW2 + 1e-15)
    assert np.all(np.abs(gq[0] - gf[0]) <= u * aW1 + 1e-15)
    assert np.all(np.abs(gq[1] - gf[1]) <= ab1 + 1e-15)
    assert np.array_equal(gq[3], gf[3])         # the b2 gradient sums unrounded dy
    # the rounding is real: the two modes are not identical
    assert not np.array_equal(gq[2], gf[2])
    # the rounded operands are bfloat16 values
    for t in trace:
        assert np.array_equal(t[4], learned.bf16(t[3])) and np.array_equal(t[6], learned.bf16(t[5]))
