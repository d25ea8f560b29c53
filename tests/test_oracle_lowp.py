"""Pins of the oracle's precision form (oracle/lowp.py) against the
published encodings (OCP E4M3, bfloat16), library conversions, exact
special cases and the quantisation error bound."""
import numpy as np
import pytest
import torch

from oracle import hausdorff, lowp, search
from oracle.prng import projection_rows


def test_e4m3_known_codes():
    vals = [0.0, 1.0, -1.0, 448.0, -448.0, 2.0 ** -6, 0.875 * 2.0 ** -6, 2.0 ** -9, 1.0625, 1.1875,
            2.0 ** -10, 3 * 2.0 ** -10, 240.0, 0.5, 1.125]
    want = [0x00, 0x38, 0xB8, 0x7E, 0xFE, 0x08, 0x07, 0x01, 0x38, 0x3A, 0x00, 0x02, 0x77, 0x30, 0x39]
    assert lowp.e4m3_bits(np.array(vals, np.float32)).tolist() == want


def test_e4m3_round_trip_and_order():
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF, 0x80)], np.uint8)
    v = lowp.e4m3_value(codes)
    assert np.array_equal(lowp.e4m3_bits(v.astype(np.float32)), codes)
    pos = np.sort(lowp.e4m3_value(np.arange(0, 0x7F, dtype=np.uint8)))
    assert np.all(np.diff(pos) > 0) and pos[-1] == 448.0
    with pytest.raises(ValueError):
        lowp.e4m3_bits(np.array([449.0], np.float32))


def test_e4m3_matches_torch_float8():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-448, 448, 20000), rng.normal(0, 0.01, 20000),
                        rng.normal(0, 2.0 ** -8, 5000)]).astype(np.float32)
    x[x == 0] = 1.0
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(lowp.e4m3_bits(x), ref)


def test_bf16_matches_torch_and_ties():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.uniform(-1, 1, 20000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(lowp.bf16_bits(x), ref)
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8], np.float32)
    assert lowp.bf16_bits(ties).tolist() == [0x3F80, 0x3F82]


def test_fp8_scale_and_exact_special_case():
    # entries in {0, +-0.25, +-0.5}: with max 0.5 the scaled values are 0, +-224, +-448, all exact
    rng = np.random.default_rng(2)
    Q = rng.choice([0.0, 0.25, -0.25, 0.5, -0.5], size=(5, 16))
    V = rng.choice([0.0, 0.25, -0.25, 0.5, -0.5], size=(7, 16))
    Q[0, 0] = V[0, 0] = 0.5
    assert lowp.fp8_scale(Q) == np.float32(0.5) / np.float32(448)
    for fmt in ("fp8", "bf16"):
        assert lowp.approx_hausdorff_sq(Q, V, fmt) == hausdorff.hausdorff_sq(Q, V)
    assert lowp.fp8_scale(np.zeros((2, 3))) == 1.0


def _grid_sets(rng, m, d):
    x = rng.normal(size=(m, d))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return np.round(x * 4096) / 4096


@pytest.mark.parametrize("fmt,rel", [("bf16", 2.0 ** -8), ("fp8", 2.0 ** -4)])
def test_approx_within_quantisation_bound(fmt, rel):
    rng = np.random.default_rng(3)
    for _ in range(20):
        Q = _grid_sets(rng, int(rng.integers(1, 20)), 64)
        V = _grid_sets(rng, int(rng.integers(1, 20)), 64)
        qq, sq = lowp.quantise(Q, fmt)
        vv, sv = lowp.quantise(V, fmt)
        eq = np.linalg.norm(Q - sq * qq, axis=1)          # per-row quantisation error
        ev = np.linalg.norm(V - sv * vv, axis=1)
        # elementwise half-ulp bound (normal range) plus the subnormal floor
        floor_q = sq * 2.0 ** -10 * np.sqrt(Q.shape[1]) if fmt == "fp8" else 0.0
        floor_v = sv * 2.0 ** -10 * np.sqrt(V.shape[1]) if fmt == "fp8" else 0.0
        assert np.all(eq <= rel * np.linalg.norm(Q, axis=1) + floor_q + 1e-12)
        assert np.all(ev <= rel * np.linalg.norm(V, axis=1) + floor_v + 1e-12)
        nq, nv = np.linalg.norm(Q, axis=1), np.linalg.norm(V, axis=1)
        nqh, nvh = np.linalg.norm(sq * qq, axis=1), np.linalg.norm(sv * vv, axis=1)
        bound = 2 * np.max(eq[:, None] * nv[None, :] + nqh[:, None] * ev[None, :])
        D = hausdorff.pairwise_sq(Q, V)
        Dh = lowp.approx_pairwise_sq(Q, V, fmt)
        assert np.max(np.abs(Dh - D)) <= bound + 1e-12
        assert abs(lowp.approx_hausdorff_sq(Q, V, fmt) - hausdorff.hausdorff_sq(Q, V)) <= bound + 1e-12


def _tiny_index():
    rng = np.random.default_rng(4)
    sizes = rng.integers(2, 9, 120)
    off = np.concatenate([[0], np.cumsum(sizes)])
    centres = rng.normal(size=(6, 32))
    topic = rng.integers(0, 6, 120)
    X = np.concatenate([_grid_sets_around(rng, centres[t], s) for t, s in zip(topic, sizes)])
    idx = projection_rows(0, 32, 256, 4)
    return search.build_index(X, off, idx, 16), X, off


def _grid_sets_around(rng, c, m):
    x = c + 0.3 * rng.normal(size=(m, c.shape[0]))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return np.round(x * 4096) / 4096


def test_search_lowp_large_margin_is_exact_search():
    ix, X, off = _tiny_index()
    Q = X[off[5]:off[6]][:3]
    ref = search.search(ix, Q, A=3, M=1, T=40, k=5)
    for fmt in ("bf16", "fp8"):
        r = lowp.search_lowp(ix, Q, A=3, M=1, T=40, k=5, fmt=fmt, margin=100.0)
        assert sorted(r["recheck"].tolist()) == sorted(r["f2_ids"].tolist())
        assert r["ids"].tolist() == ref["ids"].tolist()
        assert np.array_equal(r["h2"], ref["h2"])


def test_search_lowp_recheck_is_a_sorted_prefix_with_exact_values():
    ix, X, off = _tiny_index()
    Q = X[off[9]:off[10]]
    for fmt in ("bf16", "fp8"):
        r = lowp.search_lowp(ix, Q, A=3, M=1, T=40, k=5, fmt=fmt, margin=0.02)
        assert 5 <= len(r["recheck"]) <= len(r["f2_ids"])
        ah = dict(zip(r["f2_ids"].tolist(), r["approx_h2"].tolist()))
        kth = sorted(ah.values())[4]
        thr = lowp.recheck_threshold(kth, 0.02)
        assert all(np.float32(ah[j]) <= thr for j in r["recheck"].tolist())
        assert all(np.float32(v) > thr for j, v in ah.items() if j not in set(r["recheck"].tolist()))
        for j, h in zip(r["ids"], r["h2"]):
            assert h == hausdorff.hausdorff_sq(Q, ix.members(int(j)))


def test_recheck_selection_hand_built_margin():
    # Approximate distances (not squared) relative to the k-th (k = 3, the
    # candidate at 1.0): with a 2 % margin a candidate is re-checked when
    # its distance is at most 1.02 times the k-th.  1.015 and 1.019 are in
    # (their squares, 1.030 and 1.038, are under 1.0404), 1.0205 and 1.03
    # are out.  A threshold that scaled the squared k-th value by 1.02
    # instead of 1.02^2 would drop 1.015 and 1.019.
    base = 0.37
    rel = np.array([0.55, 0.80, 1.0, 1.015, 1.019, 1.0205, 1.03])
    ids = np.array([40, 12, 7, 3, 29, 5, 18])
    ah2 = (rel * base) ** 2
    got = lowp.select_recheck(ids, ah2, 3, 0.02)
    assert got.tolist() == [40, 12, 7, 3, 29]
    # the same values in another input order give the same selection
    perm = np.array([6, 2, 4, 0, 5, 1, 3])
    assert lowp.select_recheck(ids[perm], ah2[perm], 3, 0.02).tolist() == [40, 12, 7, 3, 29]
    # margin 0 keeps the first k and any value equal to the k-th
    assert lowp.select_recheck(ids, ah2, 3, 0.0).tolist() == [40, 12, 7]
    tie = np.array([0.1, 0.2, 0.3, 0.3, 0.4])
    assert lowp.select_recheck(np.array([1, 2, 4, 3, 5]), tie, 3, 0.0).tolist() == [1, 2, 3, 4]
    # fewer than k candidates: all of them, in order
    assert lowp.select_recheck(np.array([9, 8]), np.array([0.5, 0.2]), 3, 0.02).tolist() == [8, 9]


def test_recheck_threshold_closed_form():
    # threshold(v, m) = v (1 + m)^2 up to float32 rounding, and exactly v
    # for m = 0; increasing in the margin
    for v in (1e-6, 0.013, 0.5, 3.7, 11.0):
        assert lowp.recheck_threshold(v, 0.0) == np.float32(v)
        for m in (0.01, 0.02, 0.1, 1.0):
            t = float(lowp.recheck_threshold(v, m))
            assert abs(t - v * (1 + m) ** 2) <= 4 * np.spacing(np.float32(v * (1 + m) ** 2))
        ts = [float(lowp.recheck_threshold(v, m)) for m in (0.0, 0.01, 0.02, 0.05)]
        assert ts == sorted(ts) and len(set(ts)) == 4
