"""GPU parity of the volume solve (7-point stencil) with the FP64 oracle, and
its reduction to the image solve on a volume of identical slices."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TH = 0.1
TAU3 = synth.TAU3


def gpu3(f_np, lam, delta, iters, inner=1, tau=TAU3, pitch=None):
    import torch

    from paper_1807_11534_amd import rdseg
    D, H, W = f_np.shape
    if pitch is None:
        f = torch.from_numpy(np.ascontiguousarray(f_np)).cuda()
    else:
        ld, lds = pitch
        big = torch.full((D * lds,), float("nan"), dtype=torch.float32, device="cuda")
        f = big.as_strided((D, H, W), (lds, ld, 1))
        f.copy_(torch.from_numpy(f_np).cuda())
    u, v, p = rdseg.solve3d(f, lam, TH, tau, delta, iters, inner)
    return u.cpu().numpy(), v.cpu().numpy(), p.cpu().numpy()


def p_norm_tol(steps):
    return 1.0 + (8 + 4 * math.sqrt(steps)) * 2.0 ** -23


@pytest.mark.parametrize("shape", [(1, 9, 13), (11, 21, 37), (20, 19, 70)])
@pytest.mark.parametrize("frac", [math.inf, 0.5, 0.1])
def test_volume_matches_oracle(gpu, shape, frac):
    rng = np.random.default_rng(sum(shape))
    z = rng.normal(size=shape) * 0.3
    f = z.astype(np.float32)
    delta = frac * float(np.abs(f).max()) if math.isfinite(frac) else math.inf
    K = 40
    u, v, p = gpu3(f, 2.0, delta, K)
    ur, vr, pr = oracle.solve3(f, 2.0, TH, TAU3, delta, K)
    assert np.abs(u - ur).max() < 1e-4
    assert np.abs(v - vr).max() < 1e-4
    assert np.abs(p - pr).max() < 1e-4
    assert np.sqrt((p.astype(np.float64) ** 2).sum(axis=0)).max() <= p_norm_tol(K)


def test_volume_inner_steps_and_pitch(gpu):
    pr = synth.config_volume(24, n=3)
    f = pr.f
    delta = 0.4 * float(np.abs(f).max())
    u, v, p = gpu3(f, pr.lam, delta, 25, inner=3, pitch=(32, 32 * 27))
    ur, vr, pp = oracle.solve3(f, pr.lam, TH, TAU3, delta, 25, inner=3)
    assert np.abs(u - ur).max() < 1e-4
    assert np.abs(p - pp).max() < 1e-4


def test_identical_slices_equal_image_solve(gpu):
    """The volume kernel with identical slices gives, slice by slice, the bits
    of the temporally blocked image kernel."""
    import torch

    from paper_1807_11534_amd import rdseg
    f2 = synth.smooth_field(45, 77, seed=6, scale=1.0, noise=0.3)
    delta = 0.5 * float(np.abs(f2).max())
    f3 = np.repeat(f2[None], 5, axis=0)
    u3, v3, p3 = gpu3(f3, 2.0, delta, 33, tau=0.125)
    u2, v2, p2 = rdseg.solve(torch.from_numpy(f2).cuda(), 2.0, TH, 0.125, delta, 33,
                             tile=(16, 16), iters_per_launch=4)
    u2, v2, p2 = u2.cpu().numpy(), v2.cpu().numpy(), p2.cpu().numpy()
    for k in range(5):
        np.testing.assert_array_equal(u3[k], u2)
        np.testing.assert_array_equal(v3[k], v2)
        np.testing.assert_array_equal(p3[0][k], p2[0])
        np.testing.assert_array_equal(p3[1][k], p2[1])
    assert (p3[2] == 0).all()


def test_volume_frozen_values_and_zero_iterations(gpu):
    rng = np.random.default_rng(4)
    f = (rng.normal(size=(9, 10, 11)) * 0.5).astype(np.float32)
    u, v, p = gpu3(f, 1.0, 0.3, 0)
    h = (f < 0).astype(np.float32)
    rd = np.abs(f.astype(np.float64)) < 0.3
    np.testing.assert_array_equal(u, h)
    assert (p == 0).all()
    u, v, p = gpu3(f, 1.0, 0.3, 20)
    np.testing.assert_array_equal(u[~rd], h[~rd])
    np.testing.assert_array_equal(v[~rd], h[~rd])
    assert (p[:, ~rd] == 0).all()


def test_volume_full_size_sampled(gpu):
    """A 128^3 ellipsoid volume, compared on a sample: after K iterations a
    voxel depends only on f within 2K voxels (each iteration reaches two
    voxels: w at x + e, then div p at x - e), so the central 24^3 block equals
    the oracle's solve of the block grown by 2K + 2 voxels per side."""
    pr = synth.config_volume(128, n=6)
    f = pr.f
    delta = 0.2 * float(np.abs(f).max())
    K = 12
    u, v, p = gpu3(f, pr.lam, delta, K)
    # dependence cone: K iterations reach at most 2K voxels (two stencil
    # phases per iteration); the sub-volume grown by 2K + 2 gives exact values
    c0, c1 = 52, 76
    g0, g1 = c0 - 2 * K - 2, c1 + 2 * K + 2
    sub = np.ascontiguousarray(f[g0:g1, g0:g1, g0:g1])
    ur, vr, pp = oracle.solve3(sub, pr.lam, TH, TAU3, delta, K)
    o = c0 - g0
    assert np.abs(u[c0:c1, c0:c1, c0:c1] - ur[o:o + 24, o:o + 24, o:o + 24]).max() < 1e-4
