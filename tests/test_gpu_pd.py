"""GPU parity of the restricted primal-dual (Chambolle-Pock) solve of eq. CR
with the FP64 oracle (the restriction carried over to another solver)."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

STEP = 1.0 / math.sqrt(8.0)


def gpu_pd(f_np, lam, delta, iters, tile=None, ipl=0, pitch=None):
    import torch

    from paper_1807_11534_amd import rdseg
    H, W = f_np.shape
    if pitch is None:
        f = torch.from_numpy(np.ascontiguousarray(f_np)).cuda()
    else:
        big = torch.full((H, pitch), float("nan"), dtype=torch.float32, device="cuda")
        big[:, :W] = torch.from_numpy(f_np).cuda()
        f = big[:, :W]
    u, p = rdseg.solve_pd(f, lam, delta, iters, tile=tile, iters_per_launch=ipl)
    return u.cpu().numpy(), p.cpu().numpy()


@pytest.mark.parametrize("frac", [math.inf, 0.5, 0.2])
@pytest.mark.parametrize("shape,pitch", [((128, 128), None), ((77, 203), 256)])
def test_pd_matches_oracle(gpu, frac, shape, pitch):
    f = synth.smooth_field(*shape, seed=shape[1], scale=0.5, noise=0.3)
    delta = frac * float(np.abs(f).max()) if math.isfinite(frac) else math.inf
    K = 150
    u, p = gpu_pd(f, 3.0, delta, K, pitch=pitch)
    ur, pr = oracle.solve_pd(f, 3.0, STEP, STEP, delta, K)
    assert np.abs(u - ur).max() < 1e-4
    assert np.abs(p - pr).max() < 1e-4
    assert np.sqrt(p[0].astype(np.float64) ** 2 + p[1] ** 2).max() <= 1 + 4 * 2.0 ** -23
    A = np.abs(f.astype(np.float64)) < delta
    h = (f < 0).astype(np.float32)
    np.testing.assert_array_equal(u[~A], h[~A])


def test_pd_configurations_bitwise_identical(gpu):
    f = synth.smooth_field(150, 170, seed=2, scale=0.5, noise=0.3)
    delta = 0.4 * float(np.abs(f).max())
    ref = None
    for tile, ipl in [((16, 16), 8), ((8, 8), 16), ((32, 32), 4), ((64, 64), 8)]:
        out = gpu_pd(f, 2.0, delta, 61, tile, ipl)
        if ref is None:
            ref = out
            continue
        np.testing.assert_array_equal(out[0], ref[0])
        np.testing.assert_array_equal(out[1], ref[1])


def test_pd_two_pixel_golden(gpu):
    from tests.test_oracle_pd import golden_cases
    for f, lam, delta, want in golden_cases():
        u, _ = gpu_pd(f, lam, delta, 4000)
        np.testing.assert_allclose(u, want, rtol=0, atol=1e-5)


def test_pd_full_size_sweep_image(gpu):
    """The 1024^2 sweep image, 300 iterations at delta = 0.5 max|f|, compared
    with the oracle on the whole grid."""
    pr = synth.config2(1, 1024, 300)
    delta = 0.5 * float(np.abs(pr.f).max())
    u, p = gpu_pd(pr.f, pr.lam, delta, 300)
    ur, _ = oracle.solve_pd(pr.f, pr.lam, STEP, STEP, delta, 300)
    assert np.abs(u - ur).max() < 1e-4
    assert ((u > 0.5) != (ur > 0.5)).mean() <= 1e-4
