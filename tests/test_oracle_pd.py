"""Pins of the restricted primal-dual (Chambolle-Pock) oracle for eq. CR,
the restriction of Sec. 3 carried over to another solver as Sec. 5 proposes.

The energy and its dual are written here independently of the oracle (sparse
matrix gradient, NumPy): weak duality must hold at every iterate, the gap must
close at convergence (an optimality certificate), and hand-derived two-pixel
minimisers (tests/golden/two_pixel_cr_minimisers.txt) must be reached.  The
trajectory itself (the extrapolation step that makes the method Chambolle and
Pock's and not a plain alternation) is pinned by a dense-matrix formulation of
the published algorithm at a finite iteration count.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests.twin import grad_matrix, pd_twin

GOLD = os.path.join(os.path.dirname(__file__), "golden", "two_pixel_cr_minimisers.txt")
STEP = 1.0 / math.sqrt(8.0)   # tau = sigma, tau sigma |grad|^2 <= 1


def cr_primal(f, lam, delta, u):
    """sum over RD of |grad u~| + lambda sum over RD of f u, u~ = H(-f) off RD."""
    f = np.asarray(f, np.float32).astype(np.float64)
    A = np.abs(f) < delta
    h = (f < 0).astype(np.float64)
    ub = np.where(A, u, h)
    g = grad_matrix(*f.shape) @ ub.ravel()
    N = f.size
    return np.sqrt(g[:N] ** 2 + g[N:] ** 2)[A.ravel()].sum() + lam * (f * u)[A].sum()


def cr_dual(f, lam, delta, p):
    """min over u in [0,1]^RD of <grad u~, p> + lambda <f, u>_RD for |p| <= 1 on
    RD, p = 0 off RD: sum_RD min(0, lambda f - div p) - sum_{off RD} H(-f) div p."""
    f = np.asarray(f, np.float32).astype(np.float64)
    A = np.abs(f) < delta
    h = (f < 0).astype(np.float64)
    G = grad_matrix(*f.shape)
    d = (-G.T @ np.concatenate([p[0].ravel(), p[1].ravel()])).reshape(f.shape)
    return np.minimum(0.0, lam * f - d)[A].sum() - (h * d)[~A].sum()


def field(seed):
    return synth.smooth_field(12, 14, seed=seed, scale=0.3, noise=0.3)


@pytest.mark.parametrize("seed", [2, 3])
@pytest.mark.parametrize("frac", [math.inf, 0.5])
@pytest.mark.parametrize("lam", [2.0, 6.0])
def test_pd_duality_gap_closes(seed, frac, lam):
    f = field(seed)
    delta = frac * float(np.abs(f).max()) if math.isfinite(frac) else math.inf
    u, p = oracle.solve_pd(f, lam, STEP, STEP, delta, 200000)
    gap = cr_primal(f, lam, delta, u) - cr_dual(f, lam, delta, p)
    assert -1e-12 <= gap <= 1e-10
    assert np.sqrt(p[0] ** 2 + p[1] ** 2).max() <= 1 + 1e-14


def test_pd_weak_duality_along_the_trajectory():
    f = field(4)
    delta = 0.6 * float(np.abs(f).max())
    for K in (0, 1, 3, 10, 30, 100, 300):
        u, p = oracle.solve_pd(f, 4.0, STEP, STEP, delta, K)
        assert cr_primal(f, 4.0, delta, u) - cr_dual(f, 4.0, delta, p) >= -1e-12


def golden_cases():
    cases = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        left, right = line.split("|")
        a = left.split()
        H, W, lam, delta = int(a[0]), int(a[1]), float(a[2]), float(a[3])
        f = np.array([float(x) for x in a[4:]], np.float32).reshape(H, W)
        want = np.array([float(x) for x in right.split()]).reshape(H, W)
        cases.append((f, lam, delta, want))
    return cases


@pytest.mark.parametrize("case", range(5))
def test_pd_two_pixel_minimisers(case):
    f, lam, delta, want = golden_cases()[case]
    u, p = oracle.solve_pd(f, lam, STEP, STEP, delta, 20000)
    np.testing.assert_allclose(u, want, rtol=0, atol=1e-9)


def test_pd_frozen_and_bounds():
    f = field(5)
    delta = 0.4 * float(np.abs(f).max())
    u, p = oracle.solve_pd(f, 3.0, STEP, STEP, delta, 500)
    A = np.abs(f.astype(np.float64)) < delta
    h = (f < 0).astype(np.float64)
    np.testing.assert_array_equal(u[~A], h[~A])
    assert (p[:, ~A] == 0).all()
    assert (u >= 0).all() and (u <= 1).all()
    assert (p[0][:, -1] == 0).all() and (p[1][-1, :] == 0).all()
    u0, _ = oracle.solve_pd(f, 3.0, STEP, STEP, 0.0, 50)   # q = 0: thresholding
    np.testing.assert_array_equal(u0, h)


@pytest.mark.parametrize("shape", [(8, 8), (7, 13)])
@pytest.mark.parametrize("frac", [math.inf, 0.5])
def test_pd_matches_matrix_twin(shape, frac):
    """Mid-trajectory iterates (37 steps, far from convergence) of the oracle
    equal those of the dense-matrix formulation to rounding."""
    f = synth.smooth_field(*shape, seed=17, scale=0.3, noise=0.3)
    delta = frac * float(np.abs(f).max()) if math.isfinite(frac) else math.inf
    u, p = oracle.solve_pd(f, 3.0, STEP, 0.9 * STEP, delta, 37)
    ut, pt = pd_twin(f, 3.0, STEP, 0.9 * STEP, delta, 37)
    assert np.abs(u - ut).max() <= 1e-12
    assert np.abs(p - pt).max() <= 1e-12
