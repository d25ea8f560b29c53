"""The inequality behind the re-rank's high-plane screen, checked in exact
arithmetic on grid vectors (no GPU).

With a = 4096 x = 64 hi + lo (lo in [0, 63]) and e = lo - 31.5 on the real
coordinates (0 on padding), |a - b| >= 64 |hi_a - hi_b| - |e_a| - |e_b|.
The screen rejects a set only when this lower bound exceeds the bound for
some query row against every database vector (or the reverse), so the
inequality is all that decides whether it can ever drop a true neighbour."""
import numpy as np
import pytest


def split(a):
    hi = np.floor_divide(a, 64)
    return hi, a - 64 * hi


def lower_bound(a, b, d):
    ha, la = split(a)
    hb, lb = split(b)
    ea = np.where(np.arange(a.shape[-1]) < d, la - 31.5, 0.0)
    eb = np.where(np.arange(b.shape[-1]) < d, lb - 31.5, 0.0)
    return 64 * np.linalg.norm(ha - hb, axis=-1) - np.linalg.norm(ea, axis=-1) - np.linalg.norm(eb, axis=-1)


@pytest.mark.parametrize("d,dp", [(7, 64), (64, 64), (100, 128), (384, 384)])
def test_bound_holds_on_random_grid_vectors(d, dp):
    rng = np.random.default_rng(d)
    a = np.zeros((2000, dp), np.int64)
    b = np.zeros((2000, dp), np.int64)
    a[:, :d] = rng.integers(-4096, 4097, (2000, d))
    # b near a (the tight regime) for half the rows, independent for the rest
    b[:1000, :d] = np.clip(a[:1000, :d] + rng.integers(-70, 71, (1000, d)), -4096, 4096)
    b[1000:, :d] = rng.integers(-4096, 4097, (1000, d))
    lb = lower_bound(a, b, d)
    true = np.linalg.norm((a - b).astype(np.float64), axis=-1)
    assert (lb <= true + 1e-9).all()


def test_bound_is_tight_at_extreme_residuals():
    # lo = 0 against lo = 63 on every coordinate, same direction as 64 dh:
    # a - b = 64 dh - 63, the bound's slack is exactly what the triangle
    # inequality gives, and it never exceeds the true distance
    d = 384
    hi_a = np.full(d, 5)
    hi_b = np.full(d, 3)
    a = 64 * hi_a + 0
    b = 64 * hi_b + 63
    lb = lower_bound(a[None], b[None], d)[0]
    true = np.linalg.norm((a - b).astype(np.float64))
    assert lb <= true
    assert true - lb < 64 * np.sqrt(d)   # and it is not vacuous


def test_bound_for_identical_vectors_is_not_positive():
    d = 50
    a = np.arange(-25, 25) * 97
    lb = lower_bound(a[None], a[None], d)[0]
    assert lb <= 0.0


# ---------------------------------------------------------------------------
# The float32 evaluation of the screen, emulated step by step in numpy
# (every numpy float32 operation rounds to nearest, as the kernel's do).
# A pair is rejected when the integer h2 = |hi_a - hi_b|^2 exceeds x^2,
# x = fl(fl(fl(tb + r_a) + r_b) * (1 + 2^-21)), tb = sqrt(bound) / 64 rounded
# up and r = sqrt(es) / 128 rounded up, es = sum (2 lo - 63)^2 over the
# real coordinates.  The kernel takes the sign of h2 - x^2 from one fused
# multiply-add, which is exact; x^2 of a float32 is exact in float64.
from decimal import Decimal, getcontext

F32 = np.float32


def _sqrt32(v, ulps_down):
    s = np.sqrt(F32(v))
    for _ in range(ulps_down):
        s = np.nextafter(s, F32(0))
    return s


def screen_x(bound, es_a, es_b, ulps_down=0, bumps=True):
    """The float32 right-hand side x of the screen (kernel order).
    ulps_down models a square root one ulp low (the hardware bound)."""
    tb = F32(_sqrt32(bound, ulps_down) * F32(1.0 / 64.0))
    if bumps:
        tb = F32(tb * F32(1.0 + 2.0 ** -19))

    def r(es):
        v = F32(_sqrt32(es, ulps_down) * F32(1.0 / 128.0))
        return F32(v * F32(1.0 + 2.0 ** -20)) if bumps else v

    s = F32(F32(tb + r(es_a)) + r(es_b))
    return F32(s * F32(1.0 + 2.0 ** -21)) if bumps else s


def _largest_admissible_h2(bound, es_a, es_b):
    """floor(X^2), X = sqrt(bound)/64 + sqrt(es_a)/128 + sqrt(es_b)/128 in
    exact (60-digit) arithmetic: the largest integer h2 that a pair within
    sqrt(bound) can have (triangle inequality), so the largest that must
    never be rejected."""
    getcontext().prec = 60
    X = Decimal(int(bound)).sqrt() / 64 + Decimal(int(es_a)).sqrt() / 128 + Decimal(int(es_b)).sqrt() / 128
    return int(X * X)


def _rejects(h2, x):
    getcontext().prec = 60
    return Decimal(int(h2)) > Decimal(float(x)) ** 2


def _hard_cases(rng, d, n_res, bound_hi):
    """(bound, es_a, es_b) where X^2 lies just above an integer (the
    integer below is the tightest admissible h2), plus bounds near 0."""
    out = []
    for _ in range(n_res):
        ea = int(rng.integers(d, d * 63 * 63 + 1))
        eb = int(rng.integers(d, d * 63 * 63 + 1))
        for b in (0, 1, 2, 3, 7, 100):
            out.append((b, ea, eb))
        B = np.arange(0, bound_hi, dtype=np.float64)
        X = np.sqrt(B) / 64 + np.sqrt(ea) / 128 + np.sqrt(eb) / 128
        fr = X * X - np.floor(X * X)
        for b in B[fr < 1e-5][:20]:
            out.append((int(b), ea, eb))
    # extreme residuals: the smallest (|2 lo - 63| = 1 everywhere) and largest
    for ea, eb in ((d, d), (d * 63 * 63, d * 63 * 63), (d, d * 63 * 63)):
        for b in (0, 1, 5, 1 << 10, 1 << 20, (1 << 28) - 1):
            out.append((b, ea, eb))
    return out


@pytest.mark.parametrize("d", [64, 384, 768, 1024])
def test_float_screen_never_rejects_an_admissible_pair(d):
    rng = np.random.default_rng(1000 + d)
    for bound, ea, eb in _hard_cases(rng, d, 40, 1 << 16):
        h2 = _largest_admissible_h2(bound, ea, eb)
        for ulps in (0, 1):
            x = screen_x(bound, ea, eb, ulps_down=ulps)
            assert not _rejects(h2, x), (d, bound, ea, eb, ulps)


def test_float_screen_without_bumps_would_reject():
    # the same search finds pairs an unbumped evaluation would reject: the
    # bumps are what makes the float test conservative
    rng = np.random.default_rng(7)
    hits = 0
    for bound, ea, eb in _hard_cases(rng, 64, 60, 1 << 16):
        h2 = _largest_admissible_h2(bound, ea, eb)
        hits += _rejects(h2, screen_x(bound, ea, eb, bumps=False))
    assert hits > 0


def _screen_pair(A, B, d):
    """(h2 = |hi_A - hi_B|^2, es_A, es_B, exact D2 = |A - B|^2) of two grid
    vectors given as integers a = 4096 x."""
    ha, la = split(A)
    hb, lb = split(B)
    ea = int(((2 * la[:d] - 63) ** 2).sum())
    eb = int(((2 * lb[:d] - 63) ** 2).sum())
    return int(((ha - hb) ** 2).sum()), ea, eb, int(((A - B) ** 2).sum())


@pytest.mark.parametrize("d", [64, 384, 768, 1024])
def test_float_screen_keeps_pairs_at_their_own_distance(d):
    # near-duplicate grid vectors (distance 1e-4 .. 0.05, the regime of a
    # tiny k-th distance) and unrelated ones, each screened against a bound
    # equal to its own exact squared distance: never rejected
    rng = np.random.default_rng(2000 + d)
    for i in range(300):
        x = rng.normal(size=d)
        x /= np.linalg.norm(x)
        A = np.rint(x * 4096).astype(np.int64)
        if i % 3 == 2:
            y = rng.normal(size=d)
            y /= np.linalg.norm(y)
        else:
            y = x + rng.normal(size=d) * (10.0 ** rng.uniform(-4, -1.3)) / np.sqrt(d)
        B = np.clip(np.rint(y * 4096), -4096, 4096).astype(np.int64)
        h2, ea, eb, D2 = _screen_pair(A, B, d)
        for ulps in (0, 1):
            assert not _rejects(h2, screen_x(D2, ea, eb, ulps_down=ulps))
