"""Pins of the oracle's derivatives (reverse, tangent) and of the fitting terms.

The reverse mode is checked against the independently written tangent-linear
mode (dot-product identity) and against central finite differences of the
forward solve; the fitting terms against hand-worked values of eq. CV / eq. DS.
"""
import numpy as np
import pytest

import oracle
import synth

TH, TAU = 0.1, 0.125


def field(H, W, seed):
    return synth.smooth_field(H, W, seed, scale=0.6, noise=0.15)


@pytest.mark.parametrize("delta", [np.inf, 0.35])
def test_dot_product_identity(delta):
    """<J (df, dlam), (ubar, vbar)> == <(df, dlam), J^T (ubar, vbar)>."""
    f = field(14, 11, 1)
    rng = np.random.default_rng(5)
    df = rng.normal(size=f.shape)
    ub, vb = rng.normal(size=f.shape), rng.normal(size=f.shape)
    du, dv = oracle.tangent(f, 3.0, TH, TAU, delta, 45, df, 0.4)
    fb, lb = oracle.reverse(f, 3.0, TH, TAU, delta, 45, ub, vb)
    lhs = (du * ub).sum() + (dv * vb).sum()
    rhs = (df * fb).sum() + 0.4 * lb
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))


@pytest.mark.parametrize("delta", [np.inf, 0.35])
def test_reverse_vs_finite_differences(delta):
    """Central differences of the FP64 forward solve (domain and u0 held fixed by
    keeping perturbations away from the thresholds)."""
    H, W, K, lam = 12, 10, 30, 2.5
    f = field(H, W, 2)
    A = np.abs(f.astype(np.float64)) < delta
    rng = np.random.default_rng(6)
    target = rng.uniform(0, 1, f.shape)

    def loss(ff, ll):
        u, _, _ = oracle.solve(ff, ll, TH, TAU, delta, K)
        return ((u - target) ** 2).sum()

    u, _, _ = oracle.solve(f, lam, TH, TAU, delta, K)
    fb, lb = oracle.reverse(f, lam, TH, TAU, delta, K, 2 * (u - target))
    h = 1e-6
    fd_l = (loss(f, lam + h) - loss(f, lam - h)) / (2 * h)
    assert abs(fd_l - lb) <= 1e-6 * max(1.0, abs(fd_l))
    # per-pixel: a step of 2^-20 is exact in FP32 for these magnitudes
    hp = 2.0 ** -20
    idx = [(y, x) for y in range(H) for x in range(W)
           if A[y, x] and abs(abs(f[y, x]) - delta) > 1e-3 and abs(f[y, x]) > 1e-3]
    for (y, x) in [idx[i] for i in rng.choice(len(idx), min(8, len(idx)), replace=False)]:
        fp, fm = f.copy(), f.copy()
        fp[y, x] += np.float32(hp)
        fm[y, x] -= np.float32(hp)
        step = float(fp[y, x]) - float(fm[y, x])
        fd = (loss(fp, lam) - loss(fm, lam)) / step
        assert abs(fd - fb[y, x]) <= 1e-5 * max(1e-2, abs(fd)), (y, x, fd, fb[y, x])
    assert (fb[~A] == 0).all()


def test_fit_term_hand_values():
    """eq. CV: f = (z-c1)^2 - (z-c2)^2; eq. DS adds gamma P."""
    z = np.array([0.0, 0.5, 1.0], np.float32)
    f = oracle.fit_term(z, 0.75, 0.25)
    np.testing.assert_allclose(f, [0.5, 0.0, -0.5], atol=1e-15)
    P = np.array([0.0, 0.5, 1.0], np.float32)
    f = oracle.fit_term(z, 0.75, 0.25, gamma=2.0, P=P)
    np.testing.assert_allclose(f, [0.5, 1.0, 1.5], atol=1e-15)


def test_fit_vjp_finite_differences():
    rng = np.random.default_rng(7)
    z = rng.uniform(0, 1, 50).astype(np.float32)
    P = rng.uniform(0, 1, 50).astype(np.float32)
    fb = rng.normal(size=50)
    c1, c2, g = 0.7, 0.2, 1.5
    a, b, gg = oracle.fit_vjp(z, c1, c2, fb, P)
    h = 1e-6

    def L(c1_, c2_, g_):
        return (oracle.fit_term(z, c1_, c2_, g_, P) * fb).sum()

    assert abs((L(c1 + h, c2, g) - L(c1 - h, c2, g)) / (2 * h) - a) < 1e-7
    assert abs((L(c1, c2 + h, g) - L(c1, c2 - h, g)) / (2 * h) - b) < 1e-7
    assert abs((L(c1, c2, g + h) - L(c1, c2, g - h)) / (2 * h) - gg) < 1e-7
