"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them compares the oracle with
itself: they use hand-derived minimisers, certificates of optimality, closed
forms, symmetries, invariants, or an independent matrix formulation.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests.twin import (Twin, dense_primal_dual_split, dual_value, restricted_energy,
                        rof_dual_objective)

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TH, TAU = 0.1, 0.125


def rand_f(H, W, seed, scale=1.0):
    return synth.smooth_field(H, W, seed, scale=scale, noise=0.2)


# ---------------------------------------------------------------- operators
def test_grad_div_hand_worked():
    """Chambolle's discrete operators (end of Sec. 2.1), worked by hand on 2x3."""
    u = np.array([[1.0, 2.0, 4.0], [0.0, 3.0, 3.0]])
    gx, gy = oracle.grad(u)
    np.testing.assert_array_equal(gx, [[1, 2, 0], [3, 0, 0]])
    np.testing.assert_array_equal(gy, [[-1, 1, -1], [0, 0, 0]])
    px = np.array([[1.0, 2.0, 9.0], [3.0, 5.0, 9.0]])   # last column never used
    py = np.array([[1.0, -1.0, 2.0], [9.0, 9.0, 9.0]])  # last row never used
    d = oracle.div(px, py)
    # row 0: x-part (1, 2-1, -2), y-part (1, -1, 2); row 1: x-part (3, 5-3, -5), y-part (-1, 1, -2)
    np.testing.assert_array_equal(d, [[2, 0, 0], [2, 3, -7]])


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (9, 1), (8, 8), (13, 21)])
def test_div_is_negative_adjoint_of_grad(shape):
    rng = np.random.default_rng(3)
    u = rng.normal(size=shape)
    px, py = rng.normal(size=shape), rng.normal(size=shape)
    gx, gy = oracle.grad(u)
    lhs = (gx * px + gy * py).sum()
    rhs = -(u * oracle.div(px, py)).sum()
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


# ---------------------------------------------------------------- active set
@pytest.mark.parametrize("shape", [(1, 1), (8, 8), (13, 21), (17, 9), (40, 33)])
@pytest.mark.parametrize("delta", [-1.0, 0.0, 0.05, 0.3, np.inf])
def test_active_set_brute_force(shape, delta):
    """Sec. 3: RD = {x : -q < f(x) < q}; tiles / masks / pixel list by brute force."""
    H, W = shape
    f = rand_f(H, W, 11)
    f[0, 0] = np.nan if H * W > 1 else f[0, 0]
    out = oracle.active_set(f, delta)
    act = {(y, x) for y in range(H) for x in range(W)
           if not np.isnan(f[y, x]) and abs(float(f[y, x])) < delta}
    assert out["pixels"].tolist() == sorted(y * W + x for (y, x) in act)
    TW = (W + 7) // 8
    tiles = {}
    for (y, x) in act:
        t = (y // 8) * TW + x // 8
        tiles[t] = tiles.get(t, 0) | (1 << ((y % 8) * 8 + (x % 8)))
    assert out["tile_ids"].tolist() == sorted(tiles)
    assert [int(m) for m in out["masks"]] == [tiles[t] for t in sorted(tiles)]
    slot = out["slot_map"]
    for i, t in enumerate(sorted(tiles)):
        assert slot[t] == i
    assert (slot == -1).sum() == slot.size - len(tiles)


def test_active_set_closed_forms():
    f = rand_f(19, 26, 2)
    full = oracle.active_set(f, np.inf)
    assert full["pixels"].tolist() == list(range(19 * 26))
    assert full["tile_ids"].tolist() == list(range(3 * 4))
    # interior tile fully set, right edge tile has 2 columns, bottom edge 3 rows
    m = {int(t): int(k) for t, k in zip(full["tile_ids"], full["masks"])}
    assert m[0] == (1 << 64) - 1
    assert m[3] == sum(1 << (r * 8 + c) for r in range(8) for c in range(2))
    assert m[8] == sum(1 << (r * 8 + c) for r in range(3) for c in range(8))
    empty = oracle.active_set(f, 0.0)
    assert empty["pixels"].size == 0 and empty["tile_ids"].size == 0
    assert (empty["slot_map"] == -1).all()


# ---------------------------------------------------------------- converged
def _golden_rows():
    rows = []
    with open(os.path.join(GOLD, "two_pixel_minimisers.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(t) for t in line.split()])
    return rows


@pytest.mark.parametrize("row", _golden_rows())
def test_two_pixel_minimisers(row):
    """Hand-derived minimisers of eq. DF (box form) on 1x2, restricted as in Sec. 3."""
    f0, f1, delta, lam, theta, u0, u1, v0, v1 = row
    f = np.array([[f0, f1]], np.float32)
    u, v, _ = oracle.solve(f, lam, theta, TAU, delta, 3000)
    np.testing.assert_allclose(u.ravel(), [u0, u1], atol=1e-12)
    np.testing.assert_allclose(v.ravel(), [v0, v1], atol=1e-12)


@pytest.mark.parametrize("delta", [np.inf, 0.8, 0.35])
@pytest.mark.parametrize("lam", [0.7, 2.5])
def test_duality_gap_certificate(delta, lam):
    """The iteration's limit minimises the restricted split energy: the primal
    energy at (u, v) and the dual value at p coincide (weak duality makes the
    gap a certificate).  Sec. 2.1 eq. DF, Sec. 3 restricted systems."""
    f = rand_f(8, 8, 5, scale=0.8)
    u, v, p = oracle.solve(f, lam, TH, TAU, delta, 300000)
    P = restricted_energy(f, lam, TH, delta, u, v)
    D = dual_value(f, lam, TH, delta, p)
    assert P - D >= -1e-12
    assert P - D <= 1e-12 * max(1.0, abs(P))
    assert np.sqrt(p[0] ** 2 + p[1] ** 2).max() <= 1.0 + 1e-12



@pytest.mark.parametrize("delta", [np.inf, 0.8, 0.35, 0.1])
@pytest.mark.parametrize("lam", [0.7, 2.5])
def test_dense_projected_solve_8x8(delta, lam):
    """The limit of the iteration is the minimiser of the restricted split
    energy (Sec. 2.1 eq. DF with the restricted systems of Sec. 3): a
    brute-force dense projected primal-dual solve of that energy, to 1e-12,
    lands on the oracle's converged u and v.  The dense solve shares neither
    the algorithm nor the operators with the oracle."""
    f = rand_f(8, 8, 5, scale=0.8)
    ud, vd, _ = dense_primal_dual_split(f, lam, TH, delta)
    u, v, _ = oracle.solve(f, lam, TH, TAU, delta, 300000)
    assert np.abs(u - ud).max() <= 1e-12
    assert np.abs(v - vd).max() <= 1e-12

# ---------------------------------------------------------------- closed forms
def test_constant_f():
    """Constant f on the full domain: p stays 0 and u follows v (spec closed form)."""
    c, lam = 0.3, 2.0
    f = np.full((9, 12), c, np.float32)
    u, v, p = oracle.solve(f, lam, TH, TAU, np.inf, 50)
    assert (p == 0).all()
    assert (u == 0).all() and (v == 0).all()        # H(-c) = 0 and the clamp keeps it
    a = 0.75
    K = 4
    u, v, p = oracle.solve(f, lam, TH, TAU, np.inf, K, u0=np.full(f.shape, a))
    vk = min(max(a - TH * lam * float(np.float32(c)), 0.0), 1.0)
    for _ in range(K):
        uk, vk = vk, min(max(vk - TH * lam * float(np.float32(c)), 0.0), 1.0)
    assert (p == 0).all()
    np.testing.assert_array_equal(u, uk)
    np.testing.assert_array_equal(v, vk)


def test_heaviside_at_zero_reading():
    """The reading H(0) = 0 (the paper leaves the Heaviside function's value at
    0 open): with an empty domain u = H(-f) is 0 where f = 0, and a pixel with
    f = 0 inside RD starts from u = H(-0) = 0 and, having no data term and no
    neighbours, stays there."""
    f = np.array([[0.0, -0.5, 0.5], [-0.0, 0.0, -1.0]], np.float32)
    u, v, p = oracle.solve(f, 2.0, TH, TAU, 0.0, 10)
    np.testing.assert_array_equal(u, [[0, 1, 0], [0, 0, 1]])
    np.testing.assert_array_equal(v, u)
    u1, v1, _ = oracle.solve(np.zeros((1, 1), np.float32), 2.0, TH, TAU, 1.0, 50)
    assert u1[0, 0] == 0.0 and v1[0, 0] == 0.0

def test_large_lambda_gives_heaviside():
    """Large lambda (Sec. 1): with |div p| <= 2 + sqrt 2 and lambda*min|f| >= 4,
    v = H(-f) exactly at every iterate and the labels u > 1/2 equal H(-f)."""
    f = rand_f(24, 20, 8)
    f[np.abs(f) < 0.05] = 0.05
    lam = 4.0 / float(np.abs(f).min()) + 1.0
    for delta in [np.inf, 0.5]:
        u, v, _ = oracle.solve(f, lam, TH, TAU, delta, 60)
        h = (f < 0).astype(float)
        np.testing.assert_array_equal(v, h)
        np.testing.assert_array_equal(u > 0.5, h > 0.5)
        assert np.abs(u - h).max() <= TH * (2 + math.sqrt(2)) + 1e-12


def test_empty_domain_is_thresholding():
    """q = 0 (Sec. 3): RD empty gives u = v = H(-f), p = 0 for any K."""
    f = rand_f(15, 17, 4)
    for delta in [0.0, float(np.abs(f).min())]:
        u, v, p = oracle.solve(f, 3.0, TH, TAU, delta, 25)
        h = (f < 0).astype(float)
        np.testing.assert_array_equal(u, h)
        np.testing.assert_array_equal(v, h)
        assert (p == 0).all()


@pytest.mark.parametrize("delta", [np.inf, 0.4])
def test_complement_symmetry(delta):
    """f -> -f swaps foreground and background: (u, v, p) -> (1-u, 1-v, -p)."""
    f = rand_f(14, 11, 6)
    f[f == 0] = 1e-3
    u, v, p = oracle.solve(f, 2.0, TH, TAU, delta, 40)
    u2, v2, p2 = oracle.solve(-f, 2.0, TH, TAU, delta, 40)
    np.testing.assert_allclose(u2, 1 - u, atol=1e-13)
    np.testing.assert_allclose(v2, 1 - v, atol=1e-13)
    np.testing.assert_allclose(p2, -p, atol=1e-13)


@pytest.mark.parametrize("delta", [np.inf, 0.4])
def test_transpose_symmetry(delta):
    f = rand_f(13, 10, 7)
    u, v, p = oracle.solve(f, 2.0, TH, TAU, delta, 40)
    uT, vT, pT = oracle.solve(np.ascontiguousarray(f.T), 2.0, TH, TAU, delta, 40)
    np.testing.assert_allclose(uT, u.T, atol=1e-14)
    np.testing.assert_allclose(vT, v.T, atol=1e-14)
    np.testing.assert_allclose(pT[0], p[1].T, atol=1e-14)
    np.testing.assert_allclose(pT[1], p[0].T, atol=1e-14)


def test_resume_is_exact():
    """(u, p) is a complete state: solve(K1) then solve(K2, u, p) == solve(K1+K2)."""
    f = rand_f(12, 16, 9)
    u1, v1, p1 = oracle.solve(f, 2.0, TH, TAU, 0.5, 17)
    u2, v2, p2 = oracle.solve(f, 2.0, TH, TAU, 0.5, 13, u0=u1, p0=p1)
    u3, v3, p3 = oracle.solve(f, 2.0, TH, TAU, 0.5, 30)
    np.testing.assert_array_equal(u2, u3)
    np.testing.assert_array_equal(v2, v3)
    np.testing.assert_array_equal(p2, p3)


@pytest.mark.parametrize("delta", [np.inf, 0.5, 0.2])
def test_invariants(delta):
    """|p| <= 1 (Chambolle's step), v in [0,1], frozen pixels exact (Sec. 3)."""
    f = rand_f(21, 18, 10)
    rng = np.random.default_rng(1)
    u0 = rng.uniform(-0.5, 1.5, f.shape)
    p0 = rng.uniform(-0.7, 0.7, (2,) + f.shape)
    u, v, p = oracle.solve(f, 1.5, TH, TAU, delta, 80, u0=u0, p0=p0)
    A = np.abs(f.astype(np.float64)) < delta
    h = (f < 0).astype(float)
    assert np.sqrt(p[0] ** 2 + p[1] ** 2).max() <= 1 + 1e-15
    assert v.min() >= 0 and v.max() <= 1
    np.testing.assert_array_equal(u[~A], h[~A])
    np.testing.assert_array_equal(v[~A], h[~A])
    assert (p[:, ~A] == 0).all()
    assert (p[0][:, -1] == 0).all() and (p[1][-1, :] == 0).all()


# ---------------------------------------------------------------- twin
@pytest.mark.parametrize("shape", [(8, 8), (16, 16), (7, 13)])
@pytest.mark.parametrize("delta", [np.inf, 0.6, 0.25])
def test_matches_matrix_twin(shape, delta):
    """Equal-iteration parity with the independent matrix formulation, random starts."""
    H, W = shape
    f = rand_f(H, W, 12)
    rng = np.random.default_rng(2)
    u0 = rng.uniform(0, 1, shape)
    p0 = rng.uniform(-0.6, 0.6, (2,) + shape)
    ut, vt, pt = Twin(f, 1.7, TH, TAU, delta).run(200, u0, p0)
    u, v, p = oracle.solve(f, 1.7, TH, TAU, delta, 200, u0=u0, p0=p0)
    np.testing.assert_allclose(u, ut, atol=1e-12)
    np.testing.assert_allclose(v, vt, atol=1e-12)
    np.testing.assert_allclose(p, pt, atol=1e-12)


def test_full_domain_is_unrestricted():
    """q = 1 (Sec. 3): delta = inf is the conventional method (unmasked twin)."""
    f = rand_f(16, 16, 13)
    ut, vt, pt = Twin(f, 3.0, TH, TAU, np.inf).run(150)
    u, v, p = oracle.solve(f, 3.0, TH, TAU, np.inf, 150)
    np.testing.assert_allclose(u, ut, atol=1e-12)
    np.testing.assert_allclose(v, vt, atol=1e-12)


# ---------------------------------------------------------------- energies
@pytest.mark.parametrize("delta", [np.inf, 0.3])
def test_dual_objective_monotone(delta):
    """Chambolle's fixed point with tau <= 1/8 decreases the restricted ROF dual
    objective for fixed v (Sec. 3 fixed-point step)."""
    f = rand_f(16, 16, 14)
    rng = np.random.default_rng(4)
    v = np.where(np.abs(f) < delta, rng.uniform(0, 1, f.shape), (f < 0).astype(float))
    p = np.zeros((2,) + f.shape)
    prev = rof_dual_objective(f, TH, delta, v, p)
    for _ in range(60):
        p = oracle.dual_steps(f, v, TH, TAU, delta, 1, p0=p)
        cur = rof_dual_objective(f, TH, delta, v, p)
        assert cur <= prev + 1e-12 * max(1.0, abs(prev))
        prev = cur


def test_split_energy_monotone_exact_alternation():
    """Alternating exact minimisation (Sec. 2.1): with many inner dual steps the
    u-step is the exact restricted ROF minimiser, so E_RD never increases."""
    f = rand_f(10, 10, 15)
    delta, lam = 0.45, 2.0
    u, v, _ = oracle.solve(f, lam, TH, TAU, delta, 0)
    prev = restricted_energy(f, lam, TH, delta, u, v)
    for k in range(1, 8):
        u, v, _ = oracle.solve(f, lam, TH, TAU, delta, k, inner=4000)
        cur = restricted_energy(f, lam, TH, delta, u, v)
        assert cur <= prev + 1e-9 * max(1.0, abs(prev))
        prev = cur
