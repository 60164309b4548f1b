"""Pins of the oracle's band threshold (q -> q-hat, Sec. 3), its stopping-rule
solve and the evaluation measures E1 / E2 (Sec. 4).

The band threshold is pinned by brute force over every candidate threshold on
tiny inputs and by exact counting on larger ones; the needed count by exact
rational arithmetic (``fractions``); the stopping rule by re-measuring the
change between fixed-count solves; the measures by a hand-worked case and
their defining properties.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

TH, TAU = 0.1, 0.125


def exact_needed(q, n):
    return math.ceil(Fraction(q) * n)


# ---------------------------------------------------------------- needed count
def test_count_needed_exact():
    rng = random.Random(5)
    cases = [(0.0, 10), (1.0, 10), (0.3, 10), (0.1, 16384), (0.5, 7), (1e-300, 5),
             (5e-324, 2 ** 31 - 1), (1 - 2 ** -53, 2 ** 31 - 1), (0.7, 0), (0.25, 2 ** 31 - 1)]
    for _ in range(2000):
        cases.append((rng.random(), rng.randint(1, 2 ** 31 - 1)))
        k = rng.randint(0, 1000)
        n = rng.randint(max(1, k), 1000)
        cases.append((k / n, n))          # q n an integer up to rounding of q
    for q, n in cases:
        assert oracle.count_needed(q, n) == exact_needed(q, n), (q, n)


# ---------------------------------------------------------------- band threshold
def brute_threshold(f, q):
    """Smallest threshold t with #{|f| < t} >= ceil(q N), searched over every
    point where the count can change (0 and the double just above each |f|)."""
    a = np.abs(f.astype(np.float64)).ravel()
    k = exact_needed(q, a.size)
    cands = sorted({0.0} | {float(np.nextafter(x, np.inf)) for x in a if np.isfinite(x)})
    for t in cands:
        if int((a < t).sum()) >= k:
            return t
    return math.inf


def tiny_inputs():
    rng = np.random.default_rng(3)
    out = []
    for n in range(1, 13):
        for _ in range(6):
            shape = (1, n) if n % 2 else (2, n // 2)
            f = rng.normal(size=shape).astype(np.float32)
            if rng.random() < 0.5:          # ties
                f = np.round(f * 2) / 2
            out.append(f.astype(np.float32))
    special = np.array([[0.0, -0.0, 0.5, -0.5, np.nan, np.inf, -np.inf, 1e-45, -3.0]],
                       np.float32)
    out.append(special)
    out.append(np.full((2, 3), -0.75, np.float32))
    out.append(np.zeros((3, 3), np.float32))
    return out


@pytest.mark.parametrize("q", [0.0, 1e-9, 0.1, 0.25, 1 / 3, 0.5, 0.75, 0.9, 0.999, 1.0])
def test_band_threshold_brute_force(q):
    """Sec. 3: q-hat raised from 0 until RD holds a fraction q of the nodes."""
    for f in tiny_inputs():
        got = oracle.band_threshold(f, q)
        want = brute_threshold(f, q)
        assert got == want, (f, q, got, want)


@pytest.mark.parametrize("shape", [(64, 80), (37, 129)])
def test_band_threshold_fraction_and_minimality(shape):
    f = synth.smooth_field(*shape, seed=21, scale=1.0, noise=0.2)
    f[::7, ::5] = np.round(f[::7, ::5], 1)      # ties
    a = np.abs(f.astype(np.float64))
    N = a.size
    prev = 0.0
    for q in np.linspace(0, 1, 41):
        t = oracle.band_threshold(f, q)
        k = exact_needed(float(q), N)
        assert int((a < t).sum()) >= k
        if t > 0:
            assert int((a < np.nextafter(t, 0.0)).sum()) < k     # nothing smaller works
        assert t >= prev                                       # non-decreasing in q
        prev = t


def test_band_threshold_special_cases():
    f = synth.smooth_field(40, 50, seed=2, scale=1.0, noise=0.2)
    a = np.abs(f.astype(np.float64))
    assert oracle.band_threshold(f, 0.0) == 0.0                 # q = 0: thresholding
    t1 = oracle.band_threshold(f, 1.0)                           # q = 1: unrestricted
    assert int((a < t1).sum()) == a.size and t1 == np.nextafter(a.max(), np.inf)
    c = np.full((5, 6), 0.3, np.float32)                         # all tied
    for q in (1e-6, 0.5, 1.0):
        assert oracle.band_threshold(c, q) == np.nextafter(np.float64(np.float32(0.3)), np.inf)
    g = f.copy()
    g[0, :10] = np.nan                                           # q above the finite share
    assert oracle.band_threshold(g, 1.0) == math.inf
    # library special case: the k-th smallest |f| by selection
    for q in (0.05, 0.5, 0.95):
        k = exact_needed(q, a.size)
        kth = np.partition(a.ravel(), k - 1)[k - 1]
        assert oracle.band_threshold(f, q) == np.nextafter(kth, np.inf)


def test_band_threshold_rejects_bad_q():
    f = np.zeros((2, 2), np.float32)
    for q in (-0.1, 1.5, math.nan):
        with pytest.raises(ValueError):
            oracle.band_threshold(f, q)


# ---------------------------------------------------------------- stopping rule
def stop_problem():
    f = synth.smooth_field(24, 28, seed=8, scale=1.0, noise=0.3)
    return f, 2.0, 0.5 * float(np.abs(f).max())


@pytest.mark.parametrize("check_every", [1, 3, 8])
def test_stopping_rule_values_and_index(check_every):
    """Sec. 4: the change between consecutive iterates, in the maximum norm,
    re-measured from two fixed-count solves, and the first check below tol."""
    f, lam, delta = stop_problem()
    _, _, _, _, diffs = oracle.solve_until(f, lam, TH, TAU, delta, 64, -1.0, check_every)
    assert diffs.size == 64 // check_every
    for j, d in enumerate(diffs):
        l = (j + 1) * check_every
        u1, v1, _ = oracle.solve(f, lam, TH, TAU, delta, l)
        u0, v0, _ = oracle.solve(f, lam, TH, TAU, delta, l - 1)
        want = max(np.abs(u1 - u0).max(), np.abs(v1 - v0).max())
        assert d == want, (l, d, want)
    tol = float(np.median(diffs))
    u, v, p, done, got = oracle.solve_until(f, lam, TH, TAU, delta, 64, tol, check_every)
    first = next(j for j, d in enumerate(diffs) if d <= tol)
    assert done == (first + 1) * check_every
    np.testing.assert_array_equal(got, diffs[: first + 1])
    ur, vr, pr = oracle.solve(f, lam, TH, TAU, delta, done)
    np.testing.assert_array_equal(u, ur)
    np.testing.assert_array_equal(v, vr)
    np.testing.assert_array_equal(p, pr)


def test_stopping_rule_limits():
    f, lam, delta = stop_problem()
    assert oracle.solve_until(f, lam, TH, TAU, delta, 20, math.inf, 4)[3] == 4
    assert oracle.solve_until(f, lam, TH, TAU, delta, 20, -1.0, 4)[3] == 20
    assert oracle.solve_until(f, lam, TH, TAU, delta, 0, 1.0, 1)[3] == 0
    # empty restricted domain (Sec. 3, q = 0): nothing moves, the first check stops
    u, v, p, done, d = oracle.solve_until(f, lam, TH, TAU, 0.0, 50, 0.0, 5)
    assert done == 5 and d.tolist() == [0.0]
    np.testing.assert_array_equal(u, (f < 0).astype(np.float64))


# ---------------------------------------------------------------- E1 / E2
def test_metrics_hand_worked():
    """Sec. 4: Tanimoto coefficient of the thresholded labels and the L2 error."""
    u = np.array([[0.9, 0.2, 0.6], [0.5, 0.51, 0.0]])
    g = np.array([[1.0, 0.0, 0.4], [0.6, 0.5, 0.1]])
    # labels (> 0.5): u -> 1 0 1 / 0 1 0, g -> 1 0 0 / 1 0 0; both: 1; either: 4
    e1, e2, ni, nu = oracle.metrics(u, g)
    assert (ni, nu) == (1, 4) and e1 == 0.25
    assert abs(e2 - 0.1101) < 1e-15


def test_metrics_properties():
    rng = np.random.default_rng(0)
    u = rng.random((30, 40))
    g = rng.random((30, 40))
    assert oracle.metrics(u, u)[:2] == (1.0, 0.0)
    a, b = oracle.metrics(u, g), oracle.metrics(g, u)
    assert a[0] == b[0] and a[1] == b[1]
    assert 0.0 <= a[0] <= 1.0
    ones, zeros = np.ones((4, 4)), np.zeros((4, 4))
    assert oracle.metrics(ones, zeros)[:2] == (0.0, 16.0)
    assert oracle.metrics(zeros, zeros)[0] == 1.0        # empty union read as agreement


def test_stopping_rule_with_inner_steps():
    """With several dual steps per iteration the stopped state is the
    fixed-count solve of the same inner count."""
    f, lam, delta = stop_problem()
    _, _, _, _, d = oracle.solve_until(f, lam, TH, TAU, delta, 40, -1.0, 4, inner=3)
    tol = float(np.median(d))
    u, v, p, done, _ = oracle.solve_until(f, lam, TH, TAU, delta, 40, tol, 4, inner=3)
    ur, vr, pr = oracle.solve(f, lam, TH, TAU, delta, done, inner=3)
    np.testing.assert_array_equal(u, ur)
    np.testing.assert_array_equal(p, pr)
    u1, v1, _ = oracle.solve(f, lam, TH, TAU, delta, done - 1, inner=3)
    j = done // 4 - 1
    assert d[j] == max(np.abs(ur - u1).max(), np.abs(vr - v1).max())
