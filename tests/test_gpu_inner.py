"""GPU parity with several dual steps per outer iteration (Sec. 3: the fixed
point for p is iterated with v held; the oracle's `inner`).  Each launch then
runs iters_per_launch / inner outer iterations, since every dual step uses one
cell of the halo."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TH, TAU = 0.1, 0.125


def gpu_solve(f_np, lam, delta, iters, inner, tile=(16, 16), ipl=8):
    import torch

    from paper_1807_11534_amd import rdseg
    f = torch.from_numpy(np.ascontiguousarray(f_np)).cuda()
    u, v, p = rdseg.solve(f, lam, TH, TAU, delta, iters, tile=tile, iters_per_launch=ipl,
                          inner=inner)
    return u.cpu().numpy(), v.cpu().numpy(), p.cpu().numpy()


def p_norm_tol(steps):
    return 1.0 + (8 + 4 * math.sqrt(steps)) * 2.0 ** -23


@pytest.mark.parametrize("inner", [2, 3, 5])
@pytest.mark.parametrize("frac", [math.inf, 0.5, 0.1])
def test_inner_steps_match_oracle(gpu, inner, frac):
    f = synth.smooth_field(96, 120, seed=inner, scale=1.0, noise=0.3)
    delta = frac * float(np.abs(f).max()) if math.isfinite(frac) else math.inf
    K = 60
    u, v, p = gpu_solve(f, 2.0, delta, K, inner)
    ur, vr, pr = oracle.solve(f, 2.0, TH, TAU, delta, K, inner=inner)
    assert np.abs(u - ur).max() < 1e-4
    assert np.abs(v - vr).max() < 1e-4
    assert np.abs(p - pr).max() < 1e-4
    assert np.sqrt(p[0] ** 2 + p[1] ** 2).max() <= p_norm_tol(K * inner)
    assert ((u > 0.5) != (ur > 0.5)).mean() <= 1e-4


def test_inner_steps_configuration_invariant(gpu):
    f = synth.smooth_field(150, 170, seed=5, scale=1.0, noise=0.3)
    delta = 0.3 * float(np.abs(f).max())
    ref = None
    for tile, ipl in [((16, 16), 4), ((8, 8), 8), ((64, 64), 8), ((32, 32), 4), ((8, 8), 16),
                      ((64, 32), 4)]:
        out = gpu_solve(f, 3.0, delta, 37, 4, tile, ipl)
        if ref is None:
            ref = out
            continue
        for a, b in zip(out, ref):
            np.testing.assert_array_equal(a, b)


def test_inner_one_is_the_default(gpu):
    f = synth.smooth_field(64, 64, seed=9, scale=1.0, noise=0.3)
    a = gpu_solve(f, 2.0, 0.4, 30, 1)
    import torch

    from paper_1807_11534_amd import rdseg
    u, v, p = rdseg.solve(torch.from_numpy(f).cuda(), 2.0, TH, TAU, 0.4, 30, tile=(16, 16),
                          iters_per_launch=8)
    np.testing.assert_array_equal(a[0], u.cpu().numpy())
    np.testing.assert_array_equal(a[2], p.cpu().numpy())


def test_inner_steps_rejected_where_unsupported(gpu):
    import torch

    from paper_1807_11534_amd import rdseg
    from paper_1807_11534_amd._lib import RdsegError
    f = torch.from_numpy(synth.smooth_field(32, 32, seed=1, scale=1.0, noise=0.3)).cuda()
    with pytest.raises(RdsegError):
        rdseg.solve(f, 1.0, iters=4, tile=(16, 16), iters_per_launch=2, inner=4)
    with pytest.raises(RdsegError):
        rdseg.solve(f, 1.0, iters=4, inner=2, ckpt_every=2)


def test_inner_steps_with_stopping_rule(gpu):
    import torch

    from paper_1807_11534_amd import rdseg
    f_np = synth.smooth_field(80, 90, seed=13, scale=1.0, noise=0.3)
    delta = 0.5 * float(np.abs(f_np).max())
    f = torch.from_numpy(f_np).cuda()
    _, _, _, _, d_o = oracle.solve_until(f_np, 2.0, TH, TAU, delta, 60, -1.0, 3, inner=3)
    _, _, _, done, d = rdseg.solve_until(f, 2.0, TH, TAU, delta, 60, -1.0, 3, tile=(16, 16),
                                         iters_per_launch=8, inner=3)
    np.testing.assert_allclose(d.cpu().numpy(), d_o, rtol=0, atol=2e-4)
    tol = float(np.median(d_o))
    u, v, p, done, _ = rdseg.solve_until(f, 2.0, TH, TAU, delta, 60, tol, 3, tile=(16, 16),
                                         iters_per_launch=8, inner=3)
    n = int(done.item())
    uf, vf, pf = gpu_solve(f_np, 2.0, delta, n, 3)
    np.testing.assert_array_equal(u.cpu().numpy(), uf)
    np.testing.assert_array_equal(p.cpu().numpy(), pf)
