"""GPU parity of the convergence-driven solve (the stopping rule of Sec. 4)
and of the evaluation measures E1 / E2.

The stop is decided on the device from FP32 iterates, so its iteration can
differ from the FP64 oracle's only where the oracle's change at a check lies
within the FP32 error of the tolerance; everything else is exact: the result
equals a fixed-count solve of the reported length bit for bit, and the
measured changes follow the oracle's within twice the iterate tolerance.
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TH, TAU = 0.1, 0.125
U_TOL = 1e-4            # FP32 iterate vs FP64 oracle at equal iteration count
DIFF_TOL = 2 * U_TOL    # a change is the difference of two such iterates


def until(f_np, lam, delta, max_iters, tol, ce, tile=(16, 16), ipl=4, pitch=None, poll=True):
    import torch

    from paper_1807_11534_amd import rdseg
    H, W = f_np.shape
    if pitch is None:
        f = torch.from_numpy(np.ascontiguousarray(f_np)).cuda()
    else:
        big = torch.zeros((H, pitch), dtype=torch.float32, device="cuda")
        big[:, :W] = torch.from_numpy(f_np).cuda()
        f = big[:, :W]
    u, v, p, done, diffs = rdseg.solve_until(f, lam, TH, TAU, delta, max_iters, tol, ce,
                                             tile=tile, iters_per_launch=ipl, poll=poll)
    return (u.cpu().numpy(), v.cpu().numpy(), p.cpu().numpy(), int(done.item()),
            diffs.cpu().numpy())


def fixed(f_np, lam, delta, iters, tile=(16, 16), ipl=4):
    import torch

    from paper_1807_11534_amd import rdseg
    f = torch.from_numpy(np.ascontiguousarray(f_np)).cuda()
    u, v, p = rdseg.solve(f, lam, TH, TAU, delta, iters, tile=tile, iters_per_launch=ipl)
    return u.cpu().numpy(), v.cpu().numpy(), p.cpu().numpy()


def problem(kind):
    if kind == "c1_full":
        pr = synth.config1()
        return pr.f, pr.lam, math.inf
    pr = synth.config1()
    return pr.f, pr.lam, 0.5 * float(np.abs(pr.f).max())


@pytest.mark.parametrize("kind", ["c1_full", "c1_band"])
@pytest.mark.parametrize("ce", [1, 7, 10])
def test_stop_equals_fixed_solve_and_oracle(gpu, kind, ce):
    f, lam, delta = problem(kind)
    K = 240
    _, _, _, done_all, d_all = until(f, lam, delta, K, -1.0, ce)
    assert done_all == K and d_all.size == K // ce and (d_all > 0).all()
    # the changes follow the oracle's trajectory
    _, _, _, done_o, d_o = oracle.solve_until(f, lam, TH, TAU, delta, K, -1.0, ce)
    assert done_o == K
    np.testing.assert_allclose(d_all, d_o, rtol=0, atol=DIFF_TOL)
    # stop part-way: at the first check at or below tol, and nothing after it
    tol = float(np.sort(d_all)[d_all.size // 2])
    u, v, p, done, d = until(f, lam, delta, K, tol, ce)
    first = int(np.argmax(d_all <= tol))
    assert done == (first + 1) * ce
    np.testing.assert_array_equal(d[: first + 1], d_all[: first + 1])
    assert (d[first + 1:] == 0).all()
    uf, vf, pf = fixed(f, lam, delta, done)
    np.testing.assert_array_equal(u, uf)
    np.testing.assert_array_equal(v, vf)
    np.testing.assert_array_equal(p, pf)
    # the oracle's stop with the same tolerance agrees up to checks whose
    # change lies within the FP32 error of tol
    _, _, _, done_or, _ = oracle.solve_until(f, lam, TH, TAU, delta, K, tol, ce)
    if done_or != done:
        c = min(done, done_or) // ce - 1     # the check where the two disagree
        assert abs(d_o[c] - tol) <= DIFF_TOL, (done, done_or)
    ur, vr, _ = oracle.solve(f, lam, TH, TAU, delta, done)
    assert np.abs(u - ur).max() < U_TOL


@pytest.mark.parametrize("ce", [1, 3])
def test_poll_and_device_only_agree(gpu, ce):
    """Host polling (chunks of 2, 4, 8, ... checks) and the device-only
    schedule give the same stop and the same bits, for stops at the first
    check, inside and at the end of the first chunks, late, and never."""
    f, lam, delta = problem("c1_band")
    K = 600
    _, _, _, _, d_all = until(f, lam, delta, K, -1.0, ce, poll=False)
    picks = [math.inf, float(d_all[1]), float(d_all[2]), float(d_all[5]), float(d_all[6]),
             float(np.sort(d_all)[len(d_all) // 3]), float(d_all.min()), -1.0]
    for tol in picks:
        a = until(f, lam, delta, K, tol, ce, poll=True)
        b = until(f, lam, delta, K, tol, ce, poll=False)
        assert a[3] == b[3], tol
        for x, y in zip(a[:3], b[:3]):
            np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(a[4], b[4])


def test_stop_is_configuration_invariant(gpu):
    f, lam, delta = problem("c1_band")
    ref = None
    for tile, ipl in [((8, 8), 8), ((16, 16), 2), ((32, 32), 4), ((64, 64), 8), ((8, 8), 1)]:
        out = until(f, lam, delta, 300, 2e-3, 10, tile=tile, ipl=ipl)
        if ref is None:
            ref = out
            assert 0 < ref[3] < 300
            continue
        assert out[3] == ref[3]
        for a, b in zip(out[:3], ref[:3]):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(out[4], ref[4])


def test_stop_limits(gpu):
    f, lam, delta = problem("c1_band")
    assert until(f, lam, delta, 50, math.inf, 10)[3] == 10
    assert until(f, lam, delta, 25, -1.0, 10)[3] == 25          # checks at 10, 20 only
    u, v, p, done, d = until(f, lam, delta, 0, 1.0, 1)
    assert done == 0 and d.size == 0
    np.testing.assert_array_equal(u, fixed(f, lam, delta, 0)[0])
    # empty restricted domain: nothing moves, the first check stops the solve
    u, v, p, done, d = until(f, lam, 0.0, 100, 0.0, 5)
    assert done == 5 and d[0] == 0 and (d == 0).all()
    np.testing.assert_array_equal(u, (f < 0).astype(np.float32))


def test_stop_pitched_ragged(gpu):
    f = synth.smooth_field(83, 131, seed=12, scale=1.0, noise=0.3)
    delta = 0.4 * float(np.abs(f).max())
    _, _, _, _, d_all = until(f, 3.0, delta, 120, -1.0, 6, pitch=192)
    _, _, _, _, d_o = oracle.solve_until(f, 3.0, TH, TAU, delta, 120, -1.0, 6)
    np.testing.assert_allclose(d_all, d_o, rtol=0, atol=DIFF_TOL)
    tol = float(np.median(d_all))
    u, v, p, done, _ = until(f, 3.0, delta, 120, tol, 6, pitch=192)
    ur, vr, _ = oracle.solve(f, 3.0, TH, TAU, delta, done)
    assert np.abs(u - ur).max() < U_TOL


def test_stop_full_size_paper_tolerance(gpu):
    """The 1024^2 sweep image at delta = 0.5 max|f| with the paper's stopping
    tolerance 1e-2, checked every 10 iterations."""
    pr = synth.config2(1, 1024, 500)
    delta = 0.5 * float(np.abs(pr.f).max())
    u, v, p, done, d = until(pr.f, pr.lam, delta, 500, 1e-2, 10, tile=(64, 64), ipl=8)
    assert 0 < done <= 500
    k = done // 10
    if done < 500:
        assert d[k - 1] <= 1e-2 and (d[: k - 1] > 1e-2).all() and (d[k:] == 0).all()
    uf, vf, pf = fixed(pr.f, pr.lam, delta, done, tile=(64, 64), ipl=8)
    np.testing.assert_array_equal(u, uf)
    np.testing.assert_array_equal(p, pf)


# ---------------------------------------------------------------- E1 / E2
def gpu_metrics(u, g, eps=0.5, pitch=None):
    import torch

    from paper_1807_11534_amd import rdseg

    def dev(a):
        if pitch is None:
            return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
        big = torch.zeros((a.shape[0], pitch), dtype=torch.float32, device="cuda")
        big[:, : a.shape[1]] = torch.from_numpy(a.astype(np.float32)).cuda()
        return big[:, : a.shape[1]]
    out = rdseg.metrics(dev(u), dev(g), eps)
    return out.cpu().numpy()


@pytest.mark.parametrize("shape,pitch", [((1, 1), None), ((37, 53), 64), ((300, 257), None),
                                         ((1024, 1024), None)])
def test_metrics_match_oracle(gpu, shape, pitch):
    rng = np.random.default_rng(shape[0])
    u = rng.random(shape).astype(np.float32)
    g = rng.random(shape).astype(np.float32)
    u[rng.random(shape) < 0.05] = 0.5          # exactly at the threshold: not a label
    g[rng.random(shape) < 0.05] = 0.5
    ni, nu, e2 = gpu_metrics(u, g, pitch=pitch)
    e1o, e2o, nio, nuo = oracle.metrics(u.astype(np.float64), g.astype(np.float64))
    assert (ni, nu) == (nio, nuo)
    assert abs(e2 - e2o) <= 1e-12 * max(1.0, e2o)
    again = gpu_metrics(u, g, pitch=pitch)
    assert again.tobytes() == np.array([ni, nu, e2]).tobytes()


def test_metrics_identity_and_disjoint(gpu):
    u = np.zeros((20, 30), np.float32)
    u[5:10, 5:20] = 1
    assert gpu_metrics(u, u).tolist() == [75.0, 75.0, 0.0]
    assert gpu_metrics(u, 1 - u).tolist() == [0.0, 600.0, 600.0]
    z = np.zeros((4, 4), np.float32)
    assert gpu_metrics(z, z).tolist() == [0.0, 0.0, 0.0]
