"""Conditioning of the unrolled solve's gradient (CPU, FP64).

Where an iterate of the dual field converges with |p| < 1, grad w tends to 0
and the derivative of g/|g| is discontinuous; once |g| is at the rounding
level of w in FP32 (about 1e-7 * |w|), the direction of g -- and with it the
reverse sweep -- is fixed by rounding.  These tests measure that effect on the
64x64 boundary crop of the differentiation workload by injecting FP32-sized
noise into w of an FP64 trajectory.  They pin the cases in which an FP32
adjoint can be held to the FP64 reverse at 1e-3 and the case in which it
cannot (delta = 0.5 max|f| at 300 iterations), which the GPU parity tests
therefore run at 200 iterations.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_adjoint import boundary_crop
from tests.twin import reverse_with_w_noise

AMP = 2.0 ** -24


def crop_problem(frac, K):
    prob = synth.config5(size=512)
    sl = boundary_crop(prob)
    f = np.ascontiguousarray(prob.f[sl])
    target = prob.mask[sl].astype(np.float64)
    delta = synth.band_delta(f, frac)
    u, _, _ = oracle.solve(f, 5.0, 0.1, 0.125, delta, K)
    return f, delta, 2 * (u - target)


def test_array_reverse_matches_oracle():
    f, delta, ub = crop_problem(0.5, 60)
    g0, l0 = oracle.reverse(f, 5.0, 0.1, 0.125, delta, 60, ub)
    g1, l1 = reverse_with_w_noise(f, 5.0, 0.1, 0.125, delta, 60, ub)
    assert np.abs(g1 - g0).max() <= 1e-10 * np.abs(g0).max()
    assert abs(l1 - l0) <= 1e-10 * abs(l0)


@pytest.mark.parametrize("frac,K", [(math.inf, 300), (0.5, 200)])
def test_well_conditioned_cases(frac, K):
    f, delta, ub = crop_problem(frac, K)
    g0, _ = oracle.reverse(f, 5.0, 0.1, 0.125, delta, K, ub)
    for seed in range(3):
        g, _ = reverse_with_w_noise(f, 5.0, 0.1, 0.125, delta, K, ub,
                                    np.random.default_rng(seed), AMP)
        assert np.abs(g - g0).max() <= 1e-4 * np.abs(g0).max()


def test_ill_conditioned_case():
    f, delta, ub = crop_problem(0.5, 300)
    g0, _ = oracle.reverse(f, 5.0, 0.1, 0.125, delta, 300, ub)
    worst = 0.0
    for seed in range(6):
        g, _ = reverse_with_w_noise(f, 5.0, 0.1, 0.125, delta, 300, ub,
                                    np.random.default_rng(seed), AMP)
        worst = max(worst, np.abs(g - g0).max() / np.abs(g0).max())
    assert worst > 1e-2
