"""Batched solve over one global tile queue: bitwise equal to per-image solves
with the same tile configuration, eager and graph-replayed, and to the oracle."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def rd(gpu):
    from paper_1807_11534_amd import rdseg
    return rdseg


def make_batch(n, seed, lo=17, hi=300):
    rng = np.random.default_rng(seed)
    fs, lams, deltas = [], [], []
    for i in range(n):
        H, W = int(rng.integers(lo, hi)), int(rng.integers(lo, hi))
        f = synth.smooth_field(H, W, seed * 100 + i, noise=0.2)
        fs.append(f)
        lams.append(float(rng.uniform(1, 20)))
        frac = [math.inf, 0.5, 0.2, 0.05][i % 4]
        deltas.append(frac * float(np.abs(f).max()) if math.isfinite(frac) else math.inf)
    return fs, lams, deltas


@pytest.mark.parametrize("form", [1, 2])
@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("cfg", [((32, 32), 4), ((16, 16), 2), ((64, 64), 4)])
def test_batched_equals_single(rd, graph, cfg, form):
    """Both forms of the iterations (one persistent cooperative launch with
    grid-wide barriers, one launch per block), eager and captured in a graph,
    bitwise equal to per-image solves."""
    (tile, ipl) = cfg
    fs, lams, deltas = make_batch(11, 3)
    print(f"batched graph={graph} tile={tile} ipl={ipl} form={form}", flush=True)
    fd = [dev(f) for f in fs]
    rd.set_batched_form(form)
    try:
        bs = rd.BatchedSolver(fd, lams, deltas, 0.1, 0.125, 45, tile=tile, iters_per_launch=ipl,
                              graph=graph)
        outs = bs.run()
        if graph:
            outs = bs.run()   # a replay
    finally:
        rd.set_batched_form(2)
    for i, f in enumerate(fd):
        u, v, p = rd.solve(f, lams[i], 0.1, 0.125, deltas[i], 45, tile=tile, iters_per_launch=ipl)
        for a, b in zip(outs[i], (u, v, p)):
            np.testing.assert_array_equal(host(a), host(b))
    # oracle on two of them
    for i in (0, 5):
        uo, vo, po = oracle.solve(fs[i], lams[i], 0.1, 0.125, deltas[i], 45)
        assert np.abs(host(outs[i][0]).astype(np.float64) - uo).max() <= 1e-4
    bs.close()


def test_graph_replay_with_new_contents(rd):
    fs, lams, deltas = make_batch(6, 4)
    fd = [dev(f) for f in fs]
    bs = rd.BatchedSolver(fd, lams, deltas, 0.1, 0.125, 30, tile=(32, 32), iters_per_launch=4)
    bs.run()
    first = [host(o[0]).copy() for o in bs.out]
    # new contents in the same buffers, replay
    for i, t in enumerate(fd):
        t.copy_(dev(-fs[i]))
    outs = bs.run()
    for i in range(len(fs)):
        u, v, p = rd.solve(fd[i], lams[i], 0.1, 0.125, deltas[i], 30, tile=(32, 32),
                           iters_per_launch=4)
        np.testing.assert_array_equal(host(outs[i][0]), host(u))
        assert not np.array_equal(host(outs[i][0]), first[i]) or fs[i].size == 0
    # replays are stable
    again = [host(o[0]).copy() for o in bs.run()]
    for a, o in zip(again, outs):
        np.testing.assert_array_equal(a, host(o[0]))
    bs.close()


def test_plan_rejects_other_batch(rd):
    from paper_1807_11534_amd._lib import RdsegError
    fs, lams, deltas = make_batch(3, 5)
    fd = [dev(f) for f in fs]
    bs = rd.BatchedSolver(fd, lams, deltas, 0.1, 0.125, 10)
    bs.run()
    bs.iters = 11
    with pytest.raises(RdsegError):
        bs.run()
    bs.iters = 10
    bs.run()
    bs.close()


def test_batched_disc_rect_workload_subset(rd):
    """Eight images of the batched workload (sides 64..1024, lambda U[1,20],
    delta 0.1 max|f|, 300 iterations) against per-image solves."""
    probs = [synth.config4_image(i) for i in range(8)]
    fd = [dev(p.f) for p in probs]
    bs = rd.BatchedSolver(fd, [p.lam for p in probs], [p.delta for p in probs], 0.1, 0.125, 300)
    outs = bs.run()
    for i, p in enumerate(probs):
        u, v, pp = rd.solve(fd[i], p.lam, 0.1, 0.125, p.delta, 300, tile=(32, 32),
                            iters_per_launch=4)
        np.testing.assert_array_equal(host(outs[i][0]), host(u))
        np.testing.assert_array_equal(host(outs[i][2]), host(pp))
    bs.close()


def test_persistent_form_every_config(rd):
    """The persistent form (every block of iterations in one cooperative
    launch, grid-wide barriers) in every compiled configuration, bitwise equal
    to one launch per block.  Its grid is sized to the workgroups that are
    resident at once; a grid larger than that would leave the barriers' bounded
    waits to expire with the iterations incomplete."""
    import ctypes
    lib = rd._lib.load()
    fs, lams, deltas = make_batch(9, 7)
    fd = [dev(f) for f in fs]
    for ci in range(lib.rdseg_config_count()):
        v = [ctypes.c_int32(0) for _ in range(4)]
        lib.rdseg_config_get(ci, *[ctypes.byref(x) for x in v])
        tile, ipl = (v[0].value, v[1].value), v[2].value
        print(f"persistent form tile={tile} ipl={ipl} threads={v[3].value}", flush=True)
        outs = {}
        try:
            for form in (2, 1):
                rd.set_batched_form(form)
                bs = rd.BatchedSolver(fd, lams, deltas, 0.1, 0.125, 24, tile=tile,
                                      iters_per_launch=ipl, graph=False)
                outs[form] = [tuple(host(x) for x in o) for o in bs.run()]
        finally:
            rd.set_batched_form(2)
        for a, b in zip(outs[1], outs[2]):
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)


def test_persistent_expired_wait_marks_tiles(rd):
    """A persistent batched solve whose grid-barrier waits expire (forced from
    the host: every wait gives up at once) leaves NaN in u, v and p of its
    queued macro tiles instead of an incomplete result that could pass for a
    solution: every pixel of the images whose whole grid is RD.  The same
    batch with the default bound afterwards is bitwise the launches form."""
    fs, lams, deltas = make_batch(9, 7)
    fd = [dev(f) for f in fs]
    tile, ipl = (16, 16), 2
    print("persistent form, forced expiry", flush=True)
    try:
        rd.set_batched_form(1)
        rd.set_resident_wait(-1)
        bs = rd.BatchedSolver(fd, lams, deltas, 0.1, 0.125, 24, tile=tile, iters_per_launch=ipl,
                              graph=False)
        failed = [tuple(host(x).copy() for x in o) for o in bs.run()]
        rd.set_resident_wait(0)
        again = [tuple(host(x).copy() for x in o) for o in bs.run()]
        rd.set_batched_form(2)
        ref = [tuple(host(x).copy() for x in o) for o in bs.run()]
    finally:
        rd.set_resident_wait(0)
        rd.set_batched_form(2)
    for i, d in enumerate(deltas):
        if math.isinf(d):
            for a in failed[i]:
                assert np.isnan(a).all(), f"image {i}: a pixel of a queued tile kept a value"
    for a, b in zip(again, ref):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_batched_form_validation(rd):
    from paper_1807_11534_amd._lib import RdsegError
    with pytest.raises(RdsegError):
        rd.set_batched_form(0)
    with pytest.raises(RdsegError):
        rd.set_batched_form(3)
    rd.set_batched_form(2)


def _size_class(n):
    """The tuning cache's size class of n pixels (quarters above 4096)."""
    c = 0
    while n > 4096 and c < 12:
        n >>= 2
        c += 1
    return c


def _q_bucket(q):
    return 4 if q >= 0.5 else 3 if q >= 0.2 else 2 if q >= 0.05 else 1 if q >= 0.01 else 0


@pytest.mark.parametrize("form", [1, 2])
def test_batched_library_choice_from_cache(rd, form):
    """A batched solve that leaves the configuration to the library takes the
    tuning cache's entry for the batch's class (size class of its pixel count,
    bucket of its active fraction): eager and as a plan it runs that
    configuration and form, bitwise equal to the same batch with the
    configuration fixed, and the lookup reports it as cached."""
    fs, lams, deltas = make_batch(9, 7)
    fd = [dev(f) for f in fs]
    n_px = sum(f.size for f in fs)
    q = sum(float((np.abs(f.astype(np.float64)) < d).sum()) for f, d in zip(fs, deltas)) / n_px
    tile, ipl = (16, 16), 4
    text = ('{"version": 1, "entries": [{"size_class": %d, "q_bucket": %d, "tile_w": %d, '
            '"tile_h": %d, "iters_per_launch": %d, "components": 2, "resident": %d, '
            '"batched": 1}]}' % (_size_class(n_px), _q_bucket(q), tile[0], tile[1], ipl, form))
    print(f"batched library choice from the cache: form={form}", flush=True)
    rd.tune_cache_clear()
    try:
        rd.tune_cache_import(text)
        lib = rd.BatchedSolver(fd, lams, deltas, 0.1, 0.125, 24, tile=None, iters_per_launch=0,
                               graph=False)
        lk = lib.lookup(q)
        assert lk.cached and tuple(lk[0]) == tile and lk[1] == ipl and lk.form == form
        lib_out = [tuple(host(x) for x in o) for o in lib.run()]
        plan = rd.BatchedSolver(fd, lams, deltas, 0.1, 0.125, 24, tile=None, iters_per_launch=0,
                                graph=True)
        plan.run()
        plan_out = [tuple(host(x) for x in o) for o in plan.run()]
        plan.close()
        rd.set_batched_form(form)
        fixed = rd.BatchedSolver(fd, lams, deltas, 0.1, 0.125, 24, tile=tile,
                                 iters_per_launch=ipl, graph=False)
        fixed_out = [tuple(host(x) for x in o) for o in fixed.run()]
        for a, b, c in zip(lib_out, plan_out, fixed_out):
            for x, y, z in zip(a, b, c):
                np.testing.assert_array_equal(x, z)
                np.testing.assert_array_equal(y, z)
    finally:
        rd.set_batched_form(2)
        rd.tune_cache_clear()


@pytest.mark.skip(reason="rdseg_autotune_batched (some 80 graph captures of the batch, with "
                  "cooperative kernel nodes and fork / join events, instantiated, replayed and "
                  "destroyed) aborted the process once in this test and once under rocprofv3, "
                  "in about a dozen runs; the cause is not found, so the batched autotuner is "
                  "kept off the GPU and the benchmark takes the batch's configuration from the "
                  "committed tuning cache")
def test_batched_autotune_and_library_choice(rd):
    """rdseg_autotune_batched times every configuration and both forms on the
    batch and caches its pick under the batch's class; a solve that leaves the
    choice to the library (eager and as a plan) then runs that configuration
    and form: bitwise equal to the same batch with the configuration fixed,
    and to per-image solves."""
    fs, lams, deltas = make_batch(9, 7)
    fd = [dev(f) for f in fs]
    rd.tune_cache_clear()
    try:
        tuner = rd.BatchedSolver(fd, lams, deltas, 0.1, 0.125, 24, tile=None,
                                 iters_per_launch=0, graph=False)
        t = tuner.autotune(probe_iters=8)
        (tile, ipl), form = t, t.form
        print(f"batched autotune: tile={tile} ipl={ipl} form={form}", flush=True)
        assert form in (1, 2)
        n_px = sum(f.size for f in fs)
        q = sum(float((np.abs(f.astype(np.float64)) < d).sum()) for f, d in zip(fs, deltas)) / n_px
        lk = tuner.lookup(q)
        assert lk.cached and tuple(lk[0]) == tuple(tile) and lk[1] == ipl and lk.form == form
        lib_out = [tuple(host(x) for x in o) for o in tuner.run()]
        plan = rd.BatchedSolver(fd, lams, deltas, 0.1, 0.125, 24, tile=None, iters_per_launch=0,
                                graph=True)
        plan.run()
        plan_out = [tuple(host(x) for x in o) for o in plan.run()]
        plan.close()
        rd.set_batched_form(form)
        fixed = rd.BatchedSolver(fd, lams, deltas, 0.1, 0.125, 24, tile=tuple(tile),
                                 iters_per_launch=ipl, graph=False)
        fixed_out = [tuple(host(x) for x in o) for o in fixed.run()]
        for a, b, c in zip(lib_out, plan_out, fixed_out):
            for x, y, z in zip(a, b, c):
                np.testing.assert_array_equal(x, z)
                np.testing.assert_array_equal(y, z)
        for i in (0, 4):
            u, v, p = rd.solve(fd[i], lams[i], 0.1, 0.125, deltas[i], 24, tile=tuple(tile),
                               iters_per_launch=ipl)
            np.testing.assert_array_equal(lib_out[i][0], host(u))
    finally:
        rd.set_batched_form(2)
        rd.tune_cache_clear()
