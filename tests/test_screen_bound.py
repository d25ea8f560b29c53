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
