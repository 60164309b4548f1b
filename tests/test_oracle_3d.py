"""Pins of the oracle's volume operators and restricted solve (Sec. 5 names
3-D problems as the extension of interest; the method gains a third axis).

The volume solve is pinned to the 2-D oracle, itself pinned by optimality
certificates: a volume made of identical slices has an exactly zero z
gradient and z divergence, so every slice must reproduce the 2-D solve bit for
bit.  The z terms themselves are pinned by axis permutations (z must act as x
and y do), adjointness and a hand-worked case.
"""
import numpy as np
import pytest

import oracle
import synth

TH, TAU3 = 0.1, 1.0 / 12.0


def test_grad3_div3_hand_worked():
    z, y, x = np.mgrid[0:2, 0:2, 0:2]
    u = (4 * z + 2 * y + x).astype(np.float64)
    gx, gy, gz = oracle.grad3(u)
    np.testing.assert_array_equal(gx, np.where(x == 0, 1.0, 0.0))
    np.testing.assert_array_equal(gy, np.where(y == 0, 2.0, 0.0))
    np.testing.assert_array_equal(gz, np.where(z == 0, 4.0, 0.0))
    one = np.ones((2, 2, 2))
    d = oracle.div3(one, one, one)
    want = (np.where(x == 0, 1, -1) + np.where(y == 0, 1, -1) + np.where(z == 0, 1, -1))
    np.testing.assert_array_equal(d, want)


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 5, 7), (3, 1, 4), (4, 6, 1), (5, 6, 7)])
def test_div3_is_negative_adjoint_of_grad3(shape):
    rng = np.random.default_rng(sum(shape))
    u = rng.normal(size=shape)
    p = [rng.normal(size=shape) for _ in range(3)]
    g = oracle.grad3(u)
    lhs = sum(float((a * b).sum()) for a, b in zip(g, p))
    rhs = -float((u * oracle.div3(*p)).sum())
    assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))


@pytest.mark.parametrize("frac", [np.inf, 0.5, 0.1])
@pytest.mark.parametrize("inner", [1, 2])
def test_identical_slices_reduce_to_2d(frac, inner):
    f2 = synth.smooth_field(20, 23, seed=3, scale=1.0, noise=0.3)
    delta = frac * float(np.abs(f2).max()) if np.isfinite(frac) else np.inf
    f3 = np.repeat(f2[None], 4, axis=0)
    u3, v3, p3 = oracle.solve3(f3, 2.0, TH, 0.125, delta, 40, inner)
    u2, v2, p2 = oracle.solve(f2, 2.0, TH, 0.125, delta, 40, inner)
    for k in range(4):
        np.testing.assert_array_equal(u3[k], u2)
        np.testing.assert_array_equal(v3[k], v2)
        np.testing.assert_array_equal(p3[0][k], p2[0])
        np.testing.assert_array_equal(p3[1][k], p2[1])
    assert (p3[2] == 0).all()


def test_single_slice_is_2d():
    f2 = synth.smooth_field(17, 29, seed=8, scale=1.0, noise=0.3)
    u3, v3, p3 = oracle.solve3(f2[None], 3.0, TH, 0.125, 0.4, 30)
    u2, v2, p2 = oracle.solve(f2, 3.0, TH, 0.125, 0.4, 30)
    np.testing.assert_array_equal(u3[0], u2)
    np.testing.assert_array_equal(p3[1][0], p2[1])


@pytest.mark.parametrize("perm", [(2, 1, 0), (1, 0, 2), (0, 2, 1)])
def test_axis_permutation(perm):
    """Relabelling the axes relabels the solution: z enters as x and y do."""
    rng = np.random.default_rng(1)
    f = (rng.normal(size=(5, 6, 7)) * 0.4).astype(np.float32)
    delta = 0.5
    u, v, p = oracle.solve3(f, 2.0, TH, TAU3, delta, 50)
    ft = np.ascontiguousarray(f.transpose(perm))
    ut, vt, pt = oracle.solve3(ft, 2.0, TH, TAU3, delta, 50)
    np.testing.assert_allclose(ut, u.transpose(perm), rtol=0, atol=1e-12)
    np.testing.assert_allclose(vt, v.transpose(perm), rtol=0, atol=1e-12)
    # component along array axis a of the permuted volume = component along
    # axis perm[a] of the original; p is stored x, y, z = axes 2, 1, 0
    comp_of_axis = {2: 0, 1: 1, 0: 2}
    for a in range(3):
        src = comp_of_axis[perm[a]]
        dst = comp_of_axis[a]
        np.testing.assert_allclose(pt[dst], p[src].transpose(perm), rtol=0, atol=1e-12)


def test_volume_frozen_and_bounds():
    rng = np.random.default_rng(2)
    f = (rng.normal(size=(6, 7, 8)) * 0.5).astype(np.float32)
    u, v, p = oracle.solve3(f, 1.0, TH, TAU3, 0.3, 60)
    rd = np.abs(f.astype(np.float64)) < 0.3
    h = (f < 0).astype(np.float64)
    np.testing.assert_array_equal(u[~rd], h[~rd])
    np.testing.assert_array_equal(v[~rd], h[~rd])
    assert (p[:, ~rd] == 0).all()
    assert (v >= 0).all() and (v <= 1).all()
    assert np.sqrt((p ** 2).sum(axis=0)).max() <= 1 + 1e-12
    assert (p[0][:, :, -1] == 0).all() and (p[1][:, -1, :] == 0).all() and (p[2][-1] == 0).all()
