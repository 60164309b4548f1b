"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: active-set lists bit-exact; FP32 u within 1e-4 max-abs of the FP64
oracle at equal iteration count; thresholded labels (u > 0.5) differing on at
most 0.01 % of pixels; invariants; bitwise determinism across runs, across all
compiled tile configurations and across a resumed solve.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

U_TOL = 1e-4
LABEL_FRAC = 1e-4


def p_norm_tol(iters):
    """|p| <= 1 holds exactly in real arithmetic ((|p| + tau n) / (1 + tau n) <= 1).
    One FP32 step rounds the numerator (0.5 ulp), uses the hardware reciprocal
    and square root (<= 1 ulp each) and rounds the product (0.5 ulp): an excess
    of at most ~2 ulp of 2^-23 per step.  The next step divides the excess by
    1 + tau |g|, which is ~1 where |g| ~ 0, so over K steps the excess performs a
    random walk of K signed roundings: the bar is 8 + 4 sqrt(K) ulp."""
    return 1 + (8 + 4 * np.sqrt(iters)) * 2.0 ** -23


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rd(gpu):
    from paper_1807_11534_amd import rdseg
    return rdseg


def compare(u, v, p, uo, vo, po, f, delta, tag="", iters=500):
    u, v, p = host(u).astype(np.float64), host(v).astype(np.float64), host(p).astype(np.float64)
    err_u = np.abs(u - uo).max()
    err_v = np.abs(v - vo).max()
    lab = ((u > 0.5) != (uo > 0.5)).sum()
    assert err_u <= U_TOL, (tag, "u", err_u)
    assert err_v <= U_TOL, (tag, "v", err_v)
    assert lab <= LABEL_FRAC * u.size, (tag, "labels", lab)
    # invariants of the FP32 state
    A = np.abs(f.astype(np.float64)) < delta
    h = (f < 0).astype(np.float64)
    assert np.sqrt(p[0] ** 2 + p[1] ** 2).max() <= p_norm_tol(iters)
    assert v.min() >= 0 and v.max() <= 1
    np.testing.assert_array_equal(u[~A], h[~A])
    np.testing.assert_array_equal(v[~A], h[~A])
    assert (p[:, ~A] == 0).all()
    assert (p[0][:, -1] == 0).all() and (p[1][-1, :] == 0).all()
    return err_u, lab


# ------------------------------------------------------------ active set
@pytest.mark.parametrize("shape", [(1, 1), (8, 8), (37, 45), (64, 200), (129, 77)])
@pytest.mark.parametrize("frac", [-1.0, 0.0, 0.05, 0.3, math.inf])
def test_active_set_bit_exact(rd, shape, frac):
    H, W = shape
    f = synth.smooth_field(H, W, 21, noise=0.2)
    if H * W > 4:
        f[H // 2, W // 2] = np.nan
    delta = frac * float(np.nanmax(np.abs(f))) if math.isfinite(frac) else math.inf
    say(f"active_set {shape} delta={delta}")
    o = oracle.active_set(f, delta)
    g = rd.active_set(dev(f), delta)
    np.testing.assert_array_equal(host(g["tile_ids"]), o["tile_ids"])
    np.testing.assert_array_equal(host(g["masks"]).view(np.uint64), o["masks"])
    np.testing.assert_array_equal(host(g["slot_map"]), o["slot_map"])
    np.testing.assert_array_equal(host(g["pixels"]), o["pixels"])


def test_active_set_pitched(rd):
    """Row pitch ld > W: the same lists as the packed field."""
    f = synth.smooth_field(50, 70, 22, noise=0.2)
    big = np.zeros((50, 96), np.float32)
    big[:, :70] = f
    t = dev(big)[:, :70]
    delta = 0.25
    o = oracle.active_set(f, delta)
    g = rd.active_set(t, delta)
    np.testing.assert_array_equal(host(g["tile_ids"]), o["tile_ids"])
    np.testing.assert_array_equal(host(g["pixels"]), o["pixels"])


# ------------------------------------------------------------ solve parity
def test_plain_disc_rect_128(rd):
    """Plain method, 128x128 disc + rectangle, lambda 5, full domain, 200 iterations."""
    prob = synth.config1(seed=0)
    say("plain 128x128 K=200")
    u, v, p = rd.solve(dev(prob.f), prob.lam, prob.theta, prob.tau, math.inf, prob.iters)
    uo, vo, po = oracle.solve(prob.f, prob.lam, prob.theta, prob.tau, math.inf, prob.iters)
    compare(u, v, p, uo, vo, po, prob.f, math.inf, "c1", prob.iters)


@pytest.mark.parametrize("lam_index", [0, 1, 2])
@pytest.mark.parametrize("frac", [math.inf, 0.5, 0.2, 0.05])
def test_restricted_sweep_256(rd, lam_index, frac):
    """The restricted-domain sweep at 256^2 (lambda 1/5/20, delta fractions of max|f|)."""
    prob = synth.config2(lam_index, size=256, iters=150)
    delta = synth.band_delta(prob.f, frac)
    say(f"sweep256 lam={prob.lam} frac={frac}")
    u, v, p = rd.solve(dev(prob.f), prob.lam, prob.theta, prob.tau, delta, prob.iters)
    uo, vo, po = oracle.solve(prob.f, prob.lam, prob.theta, prob.tau, delta, prob.iters)
    compare(u, v, p, uo, vo, po, prob.f, delta, f"sweep lam={prob.lam} frac={frac}", prob.iters)


@pytest.mark.parametrize("shape", [(37, 45), (150, 203), (8, 300), (301, 9)])
def test_ragged_shapes(rd, shape):
    H, W = shape
    f = synth.smooth_field(H, W, 23, noise=0.2)
    delta = 0.4
    say(f"ragged {shape}")
    u, v, p = rd.solve(dev(f), 3.0, 0.1, 0.125, delta, 61)
    uo, vo, po = oracle.solve(f, 3.0, 0.1, 0.125, delta, 61)
    compare(u, v, p, uo, vo, po, f, delta, f"ragged {shape}", 61)


def test_all_configs_bitwise_identical(rd):
    """Every compiled (tile, iterations-per-launch) gives the same FP32 bits."""
    f = synth.smooth_field(150, 203, 24, noise=0.2)
    ft = dev(f)
    ref = None
    for (tw, th, it, nt) in rd.configs():
        say(f"config {tw}x{th} it={it} threads={nt}")
        out = [host(x) for x in rd.solve(ft, 2.0, 0.1, 0.125, 0.35, 37, tile=(tw, th),
                                         iters_per_launch=it)]
        if ref is None:
            ref = out
            uo, vo, po = oracle.solve(f, 2.0, 0.1, 0.125, 0.35, 37)
            assert np.abs(out[0] - uo).max() <= U_TOL
        else:
            for a, b in zip(out, ref):
                np.testing.assert_array_equal(a, b)



def test_autotune_restrictions(rd):
    """The autotuner returns a compiled configuration; a fixed launch depth or
    tile restricts the search to matching configurations, and a combination
    that is not compiled is an argument error.  The chosen configuration
    solves to the same bits as any other."""
    from paper_1807_11534_amd._lib import RdsegError
    f = synth.smooth_field(300, 257, 27, noise=0.2)
    ft = dev(f)
    cfgs = {(tw, th, it) for (tw, th, it, _) in rd.configs()}
    say("autotune free")
    tuned = rd.autotune(ft, 2.0, 0.1, 0.125, 0.35, 8)
    tile, ipl = tuned
    assert (tile[0], tile[1], ipl) in cfgs
    assert tuned.components in (1, 2) and tuned.resident in (1, 2)
    say("autotune resident=2")
    t2 = rd.autotune(ft, 2.0, 0.1, 0.125, 0.35, 8, resident=2)
    assert t2.resident == 2
    say("autotune iters_per_launch=8")
    tile8, ipl8 = rd.autotune(ft, 2.0, 0.1, 0.125, 0.35, 8, iters_per_launch=8)
    assert ipl8 == 8 and (tile8[0], tile8[1], 8) in cfgs
    say("autotune tile 16x16")
    t16, i16 = rd.autotune(ft, 2.0, 0.1, 0.125, 0.35, 8, tile=(16, 16))
    assert t16 == (16, 16) and (16, 16, i16) in cfgs
    with pytest.raises(RdsegError):
        rd.autotune(ft, 2.0, 0.1, 0.125, 0.35, 8, tile=(8, 8), iters_per_launch=2)
    a = [host(x) for x in rd.solve(ft, 2.0, 0.1, 0.125, 0.35, 24, tile=tile8, iters_per_launch=8)]
    b = [host(x) for x in rd.solve(ft, 2.0, 0.1, 0.125, 0.35, 24, tile=(64, 32),
                                   iters_per_launch=4)]
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_tune_cache_steers_library_choice(rd):
    """A cache entry imported as text (for this size class and active-fraction
    bucket) decides the configuration of a solve that leaves the choice to the
    library: the timing records show launches of that configuration only, and
    the result equals an explicit solve with it."""
    import json
    f = synth.smooth_field(300, 257, 31, noise=0.2)
    ft = dev(f)
    delta = 0.35
    q = float((np.abs(f.astype(np.float64)) < delta).mean())
    qb = 4 if q >= 0.5 else 3 if q >= 0.2 else 2 if q >= 0.05 else 1 if q >= 0.01 else 0
    n, cls = 300 * 257, 0
    while n > 4096 and cls < 12:
        n >>= 2
        cls += 1
    say(f"tune cache steering (class {cls}, bucket {qb})")
    try:
        for tile, ipl in [((32, 16), 2), ((16, 16), 8)]:
            rd.tune_cache_clear()
            rd.tune_cache_import(json.dumps({"version": 1, "entries": [
                {"size_class": cls, "q_bucket": qb, "tile_w": tile[0], "tile_h": tile[1],
                 "iters_per_launch": ipl, "components": 2, "resident": 2}]}))
            rd.set_resident(False)
            rd.timing_reset()
            rd.timing_enable(True)
            got = [host(x) for x in rd.solve(ft, 2.0, 0.1, 0.125, delta, 24)]
            rd.timing_enable(False)
            ci = rd.config_index(tile, ipl)
            assert rd.timing_read(ci)[1] > 0
            assert rd.timing_read(-1)[1] == rd.timing_read(ci)[1]
            ref = [host(x) for x in rd.solve(ft, 2.0, 0.1, 0.125, delta, 24, tile=tile,
                                             iters_per_launch=ipl)]
            for a, b in zip(got, ref):
                np.testing.assert_array_equal(a, b)
    finally:
        rd.timing_enable(False)
        rd.timing_reset()
        rd.set_resident(True)
        rd.tune_cache_clear()


@pytest.mark.parametrize("q_target,tile,ipl", [
    (0.004, (8, 8), 32), (0.2, (16, 16), 8), (0.8, (64, 64), 8)])
def test_untuned_choice_by_band_width(rd, q_target, tile, ipl):
    """With an empty tuning cache the library picks the configuration from the
    band's share of the image: deep launches on 8x8 tiles below 1 %, 16x16 with
    8 iterations a launch up to half the image, the 64x64 / 8 resident form
    above (all 25 of its tiles fit on the chip here).  The timing records show
    that configuration only, and the result equals an explicit solve with it."""
    f = synth.smooth_field(320, 300, 37, noise=0.2)
    ft = dev(f)
    delta = float(np.quantile(np.abs(f.astype(np.float64)), q_target))
    say(f"untuned choice at q ~ {q_target}: expect {tile} x {ipl}")
    try:
        rd.tune_cache_clear()
        rd.timing_reset()
        rd.timing_enable(True)
        got = [host(x) for x in rd.solve(ft, 2.0, 0.1, 0.125, delta, 40, components=2)]
        rd.timing_enable(False)
        ci = rd.config_index(tile, ipl)
        assert rd.timing_read(ci)[1] > 0
        assert rd.timing_read(-1)[1] == rd.timing_read(ci)[1]
        if tile == (64, 64):
            assert rd.timing_read_form(ci, 1)[1] == 1   # one resident launch
        ref = [host(x) for x in rd.solve(ft, 2.0, 0.1, 0.125, delta, 40, tile=tile,
                                         iters_per_launch=ipl, components=2)]
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
    finally:
        rd.timing_enable(False)
        rd.timing_reset()


@pytest.mark.parametrize("shape,tile,ipl,frac,iters", [
    ((1024, 1024), (64, 64), 8, math.inf, 61),
    ((1024, 1024), (64, 64), 8, 0.5, 40),
    ((700, 515), (64, 64), 8, 0.3, 33),
    ((300, 257), (64, 32), 4, 0.5, 29),
    ((64, 64), (64, 64), 8, math.inf, 5),
    ((700, 515), (32, 32), 8, 0.1, 33),
    ((1024, 1024), (32, 32), 8, 0.1, 40),
    ((512, 512), (16, 16), 8, 0.1, 27),
])
def test_resident_matches_separate_launches(rd, shape, tile, ipl, frac, iters):
    """Single-image solves whose tiles fit on the chip run as one resident
    launch; the results equal those of separate launches bit for bit, and the
    resident form is the one that ran (timing records of form 1).  The 32x32
    and 16x16 cases at 1024^2 and 512^2 have more macro tiles than fit on the
    chip at once, but their queues (the tiles of components above 64 pixels)
    do: the grid is then sized by the queue, the small components running in
    the idle workgroups (512^2) or after the tiles (1024^2)."""
    H, W = shape
    f = synth.smooth_field(H, W, 31, noise=0.2)
    delta = synth.band_delta(f, frac) if math.isfinite(frac) else math.inf
    ft = dev(f)
    say(f"resident {shape} tile={tile} ipl={ipl} frac={frac} iters={iters}")
    try:
        rd.set_resident(False)
        sep = [host(x) for x in rd.solve(ft, 3.0, 0.1, 0.125, delta, iters, tile=tile,
                                         iters_per_launch=ipl)]
        rd.set_resident(True)
        rd.timing_reset()
        rd.timing_enable(True)
        ws = rd.workspace(rd.shape_of(ft))
        res = [host(x) for x in rd.solve(ft, 3.0, 0.1, 0.125, delta, iters, tile=tile,
                                         iters_per_launch=ipl, ws=ws)]
        assert rd.solve_status(ft, ws) == 0
        ms, n, _, _ = rd.timing_read_form(-1, 1)
    finally:
        rd.timing_enable(False)
        rd.timing_reset()
        rd.set_resident(True)
    assert n == 1, "the resident form did not run"
    for a, b in zip(res, sep):
        np.testing.assert_array_equal(a, b)
    if H * W <= 300 * 257:
        uo, vo, po = oracle.solve(f, 3.0, 0.1, 0.125, delta, iters)
        assert np.abs(res[0] - uo).max() <= U_TOL
    # the barrier kind as a parameter: resident = 2 runs separate launches only
    try:
        rd.timing_reset()
        rd.timing_enable(True)
        par = [host(x) for x in rd.solve(ft, 3.0, 0.1, 0.125, delta, iters, tile=tile,
                                         iters_per_launch=ipl, resident=2)]
        n_res = rd.timing_read_form(-1, 1)[1]
        n_sep = rd.timing_read_form(-1, 0)[1]
    finally:
        rd.timing_enable(False)
        rd.timing_reset()
    assert n_res == 0 and n_sep > 0
    for a, b in zip(par, sep):
        np.testing.assert_array_equal(a, b)


def test_resident_expired_wait_is_reported(rd):
    """A resident solve whose waits for neighbouring tiles expire (forced from
    the host: every wait gives up at once) ends normally, reports
    RDSEG_ERR_TIMEOUT through rdseg_solve_status and leaves NaN in u, v and p
    of the tiles that stopped (here every tile: each has a queued
    neighbour); the next solve on the same workspace starts with a clear
    status and gives the exact result again."""
    from paper_1807_11534_amd import _lib
    f = synth.smooth_field(1024, 1024, 31, noise=0.2)
    ft = dev(f)
    ws = rd.workspace(rd.shape_of(ft))
    say("resident forced expiry 1024^2 64x64/8")
    ref = [host(x) for x in rd.solve(ft, 3.0, 0.1, 0.125, math.inf, 24, tile=(64, 64),
                                     iters_per_launch=8, resident=2, ws=ws)]
    assert rd.solve_status(ft, ws) == 0
    try:
        rd.set_resident_wait(-1)
        bad = [host(x) for x in rd.solve(ft, 3.0, 0.1, 0.125, math.inf, 24, tile=(64, 64),
                                         iters_per_launch=8, resident=1, ws=ws)]
        st = rd.solve_status(ft, ws)
    finally:
        rd.set_resident_wait(0)
    assert st == _lib.RDSEG_ERR_TIMEOUT
    assert np.isnan(bad[0]).all() and np.isnan(bad[1]).all() and np.isnan(bad[2]).all()
    good = [host(x) for x in rd.solve(ft, 3.0, 0.1, 0.125, math.inf, 24, tile=(64, 64),
                                      iters_per_launch=8, resident=1, ws=ws)]
    assert rd.solve_status(ft, ws) == 0
    for a, b in zip(good, ref):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("case", [
    dict(shape=(1024, 1024), lam=5.0, frac=0.5, iters=40, tile=(64, 64), ipl=8, inner=1),
    dict(shape=(1024, 1024), lam=1.0, frac=0.2, iters=37, tile=(16, 16), ipl=16, inner=1),
    dict(shape=(300, 257), lam=3.0, frac=0.4, iters=29, tile=(16, 16), ipl=8, inner=1),
    dict(shape=(300, 257), lam=3.0, frac=0.4, iters=21, tile=(32, 32), ipl=4, inner=2),
    dict(shape=(97, 131), lam=2.0, frac=0.3, iters=50, tile=(8, 8), ipl=8, inner=1),
    # resident solves: the workgroups left without a tile run the components
    dict(shape=(1024, 1024), lam=20.0, frac=0.5, iters=40, tile=(64, 32), ipl=4, inner=1),
    dict(shape=(300, 257), lam=3.0, frac=0.4, iters=29, tile=(64, 64), ipl=8, inner=1),
    dict(shape=(300, 257), lam=3.0, frac=0.4, iters=22, tile=(64, 32), ipl=4, inner=2),
])
def test_small_components_match_tile_path(rd, case):
    """Pixels of RD components of at most 256 pixels run whole in the component
    kernel (those of at most 64 packed into waves, the larger ones in groups of
    128 or 256 lanes with LDS exchange; in a resident solve the one-wave classes
    run in the resident kernel's workgroups that hold no tile and the groups in
    the component kernel after it); the results equal those of the tile path
    for every pixel bit for bit, and match the oracle on the smaller grids."""
    H, W = case["shape"]
    if H == 1024:
        f = synth.config2({1.0: 0, 5.0: 1, 20.0: 2}[case["lam"]], size=1024, iters=500).f
    else:
        f = synth.smooth_field(H, W, 41, noise=0.3)
    delta = synth.band_delta(f, case["frac"])
    ft = dev(f)
    say(f"components {case}")
    kw = dict(tile=case["tile"], iters_per_launch=case["ipl"], inner=case["inner"])
    try:
        rd.set_components(False)
        ref = [host(x) for x in rd.solve(ft, case["lam"], 0.1, 0.125, delta, case["iters"], **kw)]
        rd.set_components(True)
        got = [host(x) for x in rd.solve(ft, case["lam"], 0.1, 0.125, delta, case["iters"], **kw)]
    finally:
        rd.set_components(True)
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)
    if H * W <= 300 * 257:
        uo, vo, po = oracle.solve(f, case["lam"], 0.1, 0.125, delta, case["iters"],
                                  inner=case["inner"])
        assert np.abs(got[0] - uo).max() <= U_TOL

def test_determinism_and_resume(rd):
    f = synth.smooth_field(96, 130, 25, noise=0.2)
    ft = dev(f)
    say("determinism / resume")
    a = [host(x) for x in rd.solve(ft, 2.0, 0.1, 0.125, 0.4, 40, tile=(32, 32), iters_per_launch=4)]
    b = [host(x) for x in rd.solve(ft, 2.0, 0.1, 0.125, 0.4, 40, tile=(32, 32), iters_per_launch=4)]
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    u1, v1, p1 = rd.solve(ft, 2.0, 0.1, 0.125, 0.4, 23, tile=(32, 32), iters_per_launch=4)
    # resume in place: u0 is u, p0 is p
    u2, v2, p2 = rd.solve(ft, 2.0, 0.1, 0.125, 0.4, 17, u0=u1, p0=p1, tile=(16, 16),
                          iters_per_launch=2, out=(u1, v1, p1))
    for x, y in zip([host(u2), host(v2), host(p2)], a):
        np.testing.assert_array_equal(x, y)


def test_zero_iterations_is_initial_state(rd):
    f = synth.smooth_field(40, 50, 26, noise=0.2)
    u, v, p = rd.solve(dev(f), 2.0, 0.1, 0.125, 0.3, 0)
    uo, vo, po = oracle.solve(f, 2.0, 0.1, 0.125, 0.3, 0)
    np.testing.assert_array_equal(host(u), uo.astype(np.float32))
    np.testing.assert_allclose(host(v), vo, atol=1e-6)
    assert (host(p) == 0).all()


def test_closed_forms_gpu(rd):
    """Constant f, large lambda (v = H(-f) exactly), empty domain (thresholding)."""
    f = np.full((33, 41), 0.3, np.float32)
    u, v, p = rd.solve(dev(f), 2.0, 0.1, 0.125, math.inf, 30)
    assert (host(u) == 0).all() and (host(v) == 0).all() and (host(p) == 0).all()
    g = synth.smooth_field(64, 64, 27, noise=0.2)
    g[np.abs(g) < 0.05] = 0.05
    lam = 4.0 / float(np.abs(g).min()) + 1.0
    u, v, p = rd.solve(dev(g), lam, 0.1, 0.125, math.inf, 40)
    h = (g < 0).astype(np.float32)
    np.testing.assert_array_equal(host(v), h)
    np.testing.assert_array_equal(host(u) > 0.5, h > 0.5)
    u, v, p = rd.solve(dev(g), 3.0, 0.1, 0.125, 0.0, 25)
    np.testing.assert_array_equal(host(u), h)
    np.testing.assert_array_equal(host(v), h)
    assert (host(p) == 0).all()


def test_full_size_sweep_point_1024(rd):
    """1024^2, 500 iterations, lambda 5, delta 0.5 max|f|, in the benchmark's
    launch configuration, against the full oracle."""
    prob = synth.config2(1)
    delta = synth.band_delta(prob.f, 0.5)
    say("full 1024^2 K=500 frac=0.5")
    u, v, p = rd.solve(dev(prob.f), prob.lam, prob.theta, prob.tau, delta, prob.iters,
                       tile=(64, 64), iters_per_launch=4)
    uo, vo, po = oracle.solve(prob.f, prob.lam, prob.theta, prob.tau, delta, prob.iters)
    compare(u, v, p, uo, vo, po, prob.f, delta, "full1024", prob.iters)


@pytest.mark.parametrize("frac", [0.02, 0.2, 0.5])
def test_closed_tiles_match_blocked_path(rd, frac):
    """Sparse bands: tiles whose RD pixels have no RD 4-neighbour outside them
    run every iteration in one launch.  A solve that writes a checkpoint tape
    routes every tile through the temporally blocked kernel instead; the two
    must agree bitwise, and with the oracle."""
    prob = synth.config2(1, size=256, iters=120)
    delta = synth.band_delta(prob.f, frac)
    ft = dev(prob.f)
    say(f"closed tiles frac={frac}")
    for tile, ipl in [((16, 16), 8), ((64, 64), 4)]:
        a = [host(x) for x in rd.solve(ft, prob.lam, 0.1, 0.125, delta, 120, tile=tile,
                                       iters_per_launch=ipl)]
        b = [host(x) for x in rd.solve(ft, prob.lam, 0.1, 0.125, delta, 120, tile=tile,
                                       iters_per_launch=ipl, ckpt_every=120)[:3]]
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
    uo, vo, po = oracle.solve(prob.f, prob.lam, 0.1, 0.125, delta, 120)
    compare(dev(a[0]), dev(a[1]), dev(a[2]), uo, vo, po, prob.f, delta, "closed", 120)


@pytest.mark.parametrize("comps", [1, 2])
def test_single_solve_in_captured_graph(rd, comps):
    """A single-image solve captured in a graph (the small-component kernels,
    or the closed-tile kernel, on the captured stream; no resident form under
    capture) replays to the eager result bit for bit, three times, with eager
    work and synchronisation between the replays."""
    f = synth.smooth_field(300, 257, 33, noise=0.3)
    ft = dev(f)
    delta = synth.band_delta(f, 0.3)
    H, W = f.shape
    kw = dict(tile=(16, 16), iters_per_launch=8, components=comps)
    say(f"graph capture comps={comps}")
    ref = [host(x) for x in rd.solve(ft, 3.0, 0.1, 0.125, delta, 40, **kw)]
    out = (torch.empty((H, W), device="cuda"), torch.empty((H, W), device="cuda"),
           torch.empty((2, H, W), device="cuda"))
    ws = rd.workspace(rd.shape_of(ft))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):   # warm-up on the capture stream (occupancy queries)
        rd.solve(ft, 3.0, 0.1, 0.125, delta, 40, out=out, ws=ws, **kw)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rd.solve(ft, 3.0, 0.1, 0.125, delta, 40, out=out, ws=ws, **kw)
    for rep in range(3):
        for t in out:
            t.fill_(-7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [host(x) for x in out]
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        del junk


def test_release_and_reuse(rd):
    """rdseg_release frees what the library keeps for the process (side
    streams, events, the pinned buffers of timing, polling and the small
    read-backs); later calls create them again.  A component-path solve in
    separate launches (which reads its queue length back), a taped solve and
    its backward (which reads the class counts back) give the same bits
    before and after a release, and a second release in a row is harmless."""
    from paper_1807_11534_amd import _lib
    f = synth.smooth_field(300, 257, 5, noise=0.2)
    ft = dev(f)
    delta = synth.band_delta(f, 0.3)
    kw = dict(tile=(16, 16), iters_per_launch=8, components=1, resident=2)
    say("release and reuse")

    def run():
        u, v, p = rd.solve(ft, 3.0, 0.1, 0.125, delta, 40, **kw)
        out = [host(x).copy() for x in (u, v, p)]
        u2, v2, p2, tape = rd.solve(ft, 3.0, 0.1, 0.125, delta, 30, ckpt_every=10, **kw)
        gu = torch.ones_like(u2)
        gf = rd.backward(ft, 3.0, 0.1, 0.125, delta, 30, 10, tape, gu)
        out.append(host(gf[0] if isinstance(gf, tuple) else gf).copy())
        return out

    before = run()
    _lib.check(_lib.load().rdseg_release())
    _lib.check(_lib.load().rdseg_release())
    after = run()
    for a, b in zip(before, after):
        np.testing.assert_array_equal(a, b)
