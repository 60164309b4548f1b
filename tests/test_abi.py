"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and host-side validation rejects bad arguments before any launch."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rdseg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rdseg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1807_11534_amd import _lib
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if getattr(lib, n, None) is None]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1807_11534_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_status_strings(lib):
    for st in range(7):
        assert lib.rdseg_status_string(st)
    assert lib.rdseg_status_string(6) == b"a bounded on-chip wait expired"


def _solve(lib, shape, prm, f=1, u=2, v=3, p=4, ws=8, ws_bytes=1 << 40, tape=None):
    from paper_1807_11534_amd._lib import Shape
    return lib.rdseg_solve(ctypes.c_void_p(f) if f else None, Shape(*shape), ctypes.byref(prm),
                           None, None, ctypes.c_void_p(u << 32) if u else None,
                           ctypes.c_void_p(v << 32) if v else None,
                           ctypes.c_void_p(p << 32) if p else None, tape,
                           ctypes.c_void_p(ws) if ws else None, ws_bytes, None)


def _prm(**kw):
    from paper_1807_11534_amd._lib import Params
    d = dict(lambda_=1.0, theta=0.1, tau=0.125, delta=math.inf, iters=10, iters_per_launch=0,
             tile_w=0, tile_h=0, ckpt_every=0)
    d.update(kw)
    return Params(**d)


@pytest.mark.parametrize("shape,code", [((0, 5, 5), 2), ((5, 0, 5), 2), ((5, 5, 4), 2),
                                        ((1 << 16, 1 << 15, 1 << 15), 2)])
def test_bad_shapes(lib, shape, code):
    assert _solve(lib, shape, _prm()) == code


@pytest.mark.parametrize("kw", [dict(theta=0.0), dict(theta=-1.0), dict(tau=0.0),
                                dict(tau=math.nan), dict(lambda_=-1.0), dict(lambda_=math.inf),
                                dict(delta=math.nan), dict(iters=-1), dict(ckpt_every=-2),
                                dict(tile_w=64, tile_h=0, iters_per_launch=0),
                                dict(tile_w=24, tile_h=24, iters_per_launch=3)])
def test_bad_scalars(lib, kw):
    assert _solve(lib, (16, 16, 16), _prm(**kw)) == 1


def test_null_pointers_and_workspace(lib):
    assert _solve(lib, (16, 16, 16), _prm(), f=0) == 1
    assert _solve(lib, (16, 16, 16), _prm(), u=0) == 1
    assert _solve(lib, (16, 16, 16), _prm(), ws=0) == 3
    assert _solve(lib, (16, 16, 16), _prm(), ws_bytes=16) == 3
    assert _solve(lib, (16, 16, 16), _prm(ckpt_every=5)) == 5


def test_aliasing_rejected(lib):
    # v overlapping u
    assert _solve(lib, (16, 16, 16), _prm(), u=3, v=3) == 1


def test_workspace_sizes(lib):
    from paper_1807_11534_amd._lib import Shape
    s = Shape(100, 100, 128)
    n = lib.rdseg_workspace_size(ctypes.byref(s), None)
    assert n >= 4 * 4 * 100 * 128
    assert lib.rdseg_workspace_size(ctypes.byref(Shape(0, 1, 1)), None) == 0
    prm = _prm(iters=95, ckpt_every=30)
    assert lib.rdseg_tape_size(ctypes.byref(s), ctypes.byref(prm)) == 4 * 3 * 100 * 128 * 4


def test_band_threshold_validation(lib):
    from paper_1807_11534_amd._lib import Shape
    n = lib.rdseg_band_workspace_size()
    assert 8192 <= n <= 16384
    fp, out, ws = ctypes.c_void_p(1 << 32), ctypes.c_void_p(2 << 32), ctypes.c_void_p(3 << 32)
    sh = Shape(16, 16, 16)
    for q in (-0.1, 1.0000001, math.nan, math.inf):
        assert lib.rdseg_band_threshold(fp, sh, q, out, ws, n, None) == 1
    assert lib.rdseg_band_threshold(None, sh, 0.5, out, ws, n, None) == 1
    assert lib.rdseg_band_threshold(fp, sh, 0.5, None, ws, n, None) == 1
    assert lib.rdseg_band_threshold(fp, sh, 0.5, out, None, n, None) == 3
    assert lib.rdseg_band_threshold(fp, sh, 0.5, out, ws, n - 1, None) == 3
    assert lib.rdseg_band_threshold(fp, Shape(16, 16, 8), 0.5, out, ws, n, None) == 2


def test_solve_until_validation(lib):
    from paper_1807_11534_amd._lib import Shape
    sh = Shape(16, 16, 16)
    P = lambda a: ctypes.c_void_p(a << 32)

    def call(prm, tol=1e-2, ce=1, done=P(9), diffs=P(10)):
        return lib.rdseg_solve_until(P(1), sh, ctypes.byref(prm), tol, ce, 0, None, None, P(2),
                                     P(3), P(4), done, diffs, P(8), 1 << 40, None)
    assert call(_prm(), tol=math.nan) == 1
    assert call(_prm(), ce=0) == 1
    assert call(_prm(ckpt_every=5)) == 1
    assert call(_prm(), done=None) == 1
    assert call(_prm(iters=10), ce=3, diffs=None) == 1
    assert call(_prm(theta=0.0)) == 1
    assert lib.rdseg_solve_until(P(1), sh, None, 1e-2, 1, 0, None, None, P(2), P(3), P(4), P(9),
                                 P(10), P(8), 1 << 40, None) == 1


def test_metrics_validation(lib):
    from paper_1807_11534_amd._lib import Shape
    n = lib.rdseg_metrics_workspace_size()
    assert n >= 1024 * 3 * 8
    P = lambda a: ctypes.c_void_p(a << 32)
    sh = Shape(16, 16, 16)
    assert lib.rdseg_metrics(None, P(2), sh, 0.5, P(3), P(4), n, None) == 1
    assert lib.rdseg_metrics(P(1), None, sh, 0.5, P(3), P(4), n, None) == 1
    assert lib.rdseg_metrics(P(1), P(2), sh, 0.5, None, P(4), n, None) == 1
    assert lib.rdseg_metrics(P(1), P(2), sh, math.nan, P(3), P(4), n, None) == 1
    assert lib.rdseg_metrics(P(1), P(2), sh, 0.5, P(3), P(4), n - 1, None) == 3
    assert lib.rdseg_metrics(P(1), P(2), Shape(0, 16, 16), 0.5, P(3), P(4), n, None) == 2


def test_components_choice_validation(lib):
    assert _solve(lib, (16, 16, 16), _prm(components=-1)) == 1
    assert _solve(lib, (16, 16, 16), _prm(components=3)) == 1


def test_barrier_choice_validation(lib):
    assert _solve(lib, (16, 16, 16), _prm(resident=-1)) == 1
    assert _solve(lib, (16, 16, 16), _prm(resident=3)) == 1


def test_inner_steps_validation(lib):
    assert _solve(lib, (16, 16, 16), _prm(inner=-1)) == 1
    assert _solve(lib, (16, 16, 16), _prm(inner=17)) == 1
    tape = ctypes.c_void_p(7 << 32)
    assert _solve(lib, (16, 16, 16), _prm(inner=2, ckpt_every=5), tape=tape) == 1
    # an explicit configuration whose halo holds fewer dual steps than inner
    assert _solve(lib, (16, 16, 16), _prm(inner=4, tile_w=16, tile_h=16, iters_per_launch=2)) == 1


def test_volume_validation(lib):
    from paper_1807_11534_amd._lib import Shape3
    P = lambda a: ctypes.c_void_p(a << 32)
    assert lib.rdseg_workspace_size3(ctypes.byref(Shape3(4, 5, 6, 6, 30))) > 0
    assert lib.rdseg_workspace_size3(ctypes.byref(Shape3(4, 5, 6, 6, 29))) == 0

    def call(sh, prm, f=P(1)):
        return lib.rdseg_solve3d(f, sh, ctypes.byref(prm), None, None, P(2), P(3), P(4), P(8),
                                 1 << 40, None)
    ok = Shape3(4, 5, 6, 6, 30)
    assert call(Shape3(0, 5, 6, 6, 30), _prm()) == 2
    assert call(Shape3(4, 5, 6, 5, 30), _prm()) == 2
    assert call(Shape3(1 << 12, 1 << 10, 1 << 10, 1 << 10, 1 << 20), _prm()) == 2
    assert call(ok, _prm(theta=0.0)) == 1
    assert call(ok, _prm(tile_w=8, tile_h=8, iters_per_launch=1)) == 1
    assert call(ok, _prm(ckpt_every=4)) == 1
    assert call(ok, _prm(inner=17)) == 1
    assert call(ok, _prm(), f=None) == 1
    assert lib.rdseg_solve3d(P(1), ok, ctypes.byref(_prm()), None, None, P(2), P(3), P(4), P(8),
                             16, None) == 3


def test_primal_dual_validation(lib):
    from paper_1807_11534_amd._lib import PdParams, Shape
    P = lambda a: ctypes.c_void_p(a << 32)
    sh = Shape(16, 16, 16)
    n = lib.rdseg_pd_workspace_size(ctypes.byref(sh))
    assert n > lib.rdseg_workspace_size(ctypes.byref(sh), None)

    def call(**kw):
        d = dict(lambda_=1.0, tau=0.35, sigma=0.35, delta=math.inf, iters=10, iters_per_launch=0,
                 tile_w=0, tile_h=0)
        d.update(kw)
        prm = PdParams(**d)
        return lib.rdseg_solve_pd(P(1), sh, ctypes.byref(prm), None, None, P(2), P(3), P(8), n,
                                  None)
    for kw in (dict(tau=0.0), dict(sigma=-1.0), dict(lambda_=math.nan), dict(delta=math.nan),
               dict(iters=-1), dict(tile_w=24, tile_h=24, iters_per_launch=3)):
        assert call(**kw) == 1, kw
    prm = PdParams(1.0, 0.35, 0.35, math.inf, 10, 0, 0, 0)
    assert lib.rdseg_solve_pd(P(1), sh, ctypes.byref(prm), None, None, P(2), P(3), P(8), 16,
                              None) == 3
    assert lib.rdseg_solve_pd(P(1), sh, ctypes.byref(prm), None, None, P(1), P(3), P(8), n,
                              None) == 1   # u aliases f


def test_tune_cache_text_round_trip():
    """The autotuner's cache as JSON text: export, clear, import, export again
    (host only: no GPU call)."""
    import json

    from paper_1807_11534_amd import rdseg
    rdseg.tune_cache_clear()
    assert json.loads(rdseg.tune_cache_export()) == {"version": 1, "entries": []}
    entries = [
        {"size_class": 4, "q_bucket": 4, "tile_w": 64, "tile_h": 64, "iters_per_launch": 8,
         "components": 2, "resident": 1},
        {"size_class": 4, "q_bucket": 1, "tile_w": 16, "tile_h": 16, "iters_per_launch": 16,
         "components": 1, "resident": 2},
        {"size_class": 6, "q_bucket": 0, "tile_w": 8, "tile_h": 8, "iters_per_launch": 32,
         "components": 2, "resident": 1},
    ]
    rdseg.tune_cache_import(json.dumps({"version": 1, "entries": entries}))
    got = json.loads(rdseg.tune_cache_export())
    key = lambda e: (e["size_class"], e["q_bucket"])
    assert sorted(got["entries"], key=key) == sorted(entries, key=key)
    # a later entry with the same key replaces the earlier one
    repl = dict(entries[0], tile_w=32, tile_h=32)
    rdseg.tune_cache_import(json.dumps({"entries": [repl], "version": 1}))
    got = {key(e): e for e in json.loads(rdseg.tune_cache_export())["entries"]}
    assert got[(4, 4)] == repl and len(got) == 3
    rdseg.tune_cache_clear()
    assert json.loads(rdseg.tune_cache_export())["entries"] == []


@pytest.mark.parametrize("text", [
    "",
    "{}",
    '{"version": 2, "entries": []}',
    '{"version": 1}',
    '{"version": 1, "entries": [{"size_class": 4, "q_bucket": 4, "tile_w": 64, "tile_h": 64, '
    '"iters_per_launch": 8, "components": 1}]}',
    '{"version": 1, "entries": [{"size_class": 4, "q_bucket": 5, "tile_w": 64, "tile_h": 64, '
    '"iters_per_launch": 8, "components": 1, "resident": 1}]}',
    '{"version": 1, "entries": [{"size_class": 4, "q_bucket": 4, "tile_w": 48, "tile_h": 64, '
    '"iters_per_launch": 8, "components": 1, "resident": 1}]}',
    '{"version": 1, "entries": [{"size_class": 4, "q_bucket": 4, "tile_w": 64, "tile_h": 64, '
    '"iters_per_launch": 8, "components": 3, "resident": 1}]}',
    '{"version": 1, "entries": [{"size_class": 4, "q_bucket": 4, "tile_w": 64, "tile_h": 64, '
    '"iters_per_launch": 8, "components": 1, "resident": 0}]}',
    '{"version": 1, "entries": []} trailing',
    '{"version": 1, "entries": [], "extra": 1}',
])
def test_tune_cache_rejects_bad_text(text):
    from paper_1807_11534_amd import rdseg
    from paper_1807_11534_amd._lib import RdsegError
    rdseg.tune_cache_clear()
    rdseg.tune_cache_import('{"version": 1, "entries": [{"size_class": 1, "q_bucket": 0, '
                            '"tile_w": 8, "tile_h": 8, "iters_per_launch": 8, "components": 2, '
                            '"resident": 2}]}')
    before = rdseg.tune_cache_export()
    with pytest.raises(RdsegError):
        rdseg.tune_cache_import(text)
    assert rdseg.tune_cache_export() == before   # nothing merged
    rdseg.tune_cache_clear()


def test_tune_cache_export_needs_room(lib):
    n = ctypes.c_size_t(0)
    assert lib.rdseg_tune_cache_export(None, 0, ctypes.byref(n)) == 1
    assert n.value > 10
    buf = ctypes.create_string_buffer(n.value - 1)
    assert lib.rdseg_tune_cache_export(buf, n.value - 1, ctypes.byref(n)) == 1
    buf = ctypes.create_string_buffer(n.value)
    assert lib.rdseg_tune_cache_export(buf, n.value, ctypes.byref(n)) == 0


def test_noalloc_validation_before_any_gpu_call(lib):
    """rdseg_solve_noalloc rejects, on the host and before touching the GPU,
    an image whose workspace exceeds its scratch array (RDSEG_ERR_WORKSPACE)
    and a request for a tape (RDSEG_ERR_ARG)."""
    from paper_1807_11534_amd._lib import Shape

    def call(shape, prm):
        return lib.rdseg_solve_noalloc(ctypes.c_void_p(8), Shape(*shape), ctypes.byref(prm),
                                       None, None, ctypes.c_void_p(1 << 32),
                                       ctypes.c_void_p(2 << 32), ctypes.c_void_p(3 << 32), None)

    big = (2048, 2048, 2048)
    assert lib.rdseg_workspace_size(ctypes.byref(Shape(*big)), None) > (64 << 20)
    assert call(big, _prm()) == 3
    assert b"scratch array" in lib.rdseg_last_error()
    assert call((64, 64, 64), _prm(ckpt_every=5)) == 1
    assert call((0, 64, 64), _prm()) == 2
    # the largest benchmark image fits
    assert lib.rdseg_workspace_size(ctypes.byref(Shape(1024, 1024, 1024)), None) <= (64 << 20)


def test_tune_lookup_reads_the_cache():
    """rdseg_tune_lookup returns the cache entry of (size class, q bucket) for
    a shape and active fraction, and reports when it has none (host only)."""
    import json

    from paper_1807_11534_amd import rdseg
    rdseg.tune_cache_clear()
    entries = [
        {"size_class": 4, "q_bucket": 3, "tile_w": 32, "tile_h": 32, "iters_per_launch": 8,
         "components": 1, "resident": 2},
        {"size_class": 4, "q_bucket": 0, "tile_w": 8, "tile_h": 8, "iters_per_launch": 32,
         "components": 2, "resident": 1},
    ]
    rdseg.tune_cache_import(json.dumps({"version": 1, "entries": entries}))
    # 1024^2 is size class 4; q = 0.42 lies in bucket 3 ([0.2, 0.5)), 0.004 in bucket 0
    t = rdseg.tune_lookup((1024, 1024), 0.42)
    assert (t, t.components, t.resident, t.cached) == (((32, 32), 8), 1, 2, True)
    t = rdseg.tune_lookup((1024, 1024), 0.004)
    assert (t, t.components, t.resident, t.cached) == (((8, 8), 32), 2, 1, True)
    t = rdseg.tune_lookup((1024, 1024), 0.03)   # bucket 1: no entry, the fixed choice
    assert not t.cached and (t.components, t.resident) == (0, 0)
    assert t == ((16, 16), 8)
    from paper_1807_11534_amd._lib import RdsegError
    with pytest.raises(RdsegError):
        rdseg.tune_lookup((1024, 1024), 1.5)
    rdseg.tune_cache_clear()


def _fake_batch(shapes):
    from paper_1807_11534_amd._lib import Image, Shape
    arr = (Image * len(shapes))()
    for i, (H, W) in enumerate(shapes):
        base = (i + 1) << 36
        arr[i] = Image(base, base + (1 << 32), base + (2 << 32), base + (3 << 32),
                       Shape(H, W, W), 5.0, 1.0)
    return arr


def test_batched_cache_entries_and_lookup(lib):
    """Batched entries of the tuning cache ("batched": 1) round-trip through the
    text and are what rdseg_batched_lookup returns for a batch of that class
    (size class of its total pixel count, bucket of its active fraction); a
    single-image entry of the same class and bucket is a different key (host
    only)."""
    import json

    from paper_1807_11534_amd import rdseg
    rdseg.tune_cache_clear()
    shapes = [(512, 512)] * 4 + [(256, 1024)] * 4   # 2^21 pixels: size class 5
    arr = _fake_batch(shapes)
    entries = [
        {"size_class": 5, "q_bucket": 0, "tile_w": 16, "tile_h": 16, "iters_per_launch": 16,
         "components": 2, "resident": 1, "batched": 1},
        {"size_class": 5, "q_bucket": 0, "tile_w": 8, "tile_h": 8, "iters_per_launch": 32,
         "components": 2, "resident": 2},
    ]
    rdseg.tune_cache_import(json.dumps({"version": 1, "entries": entries}))
    got = json.loads(rdseg.tune_cache_export())["entries"]
    assert sorted(got, key=lambda e: e.get("batched", 0)) == [entries[1], entries[0]]
    v = [ctypes.c_int32(0) for _ in range(5)]
    assert lib.rdseg_batched_lookup(arr, len(shapes), 0.001, *[ctypes.byref(x) for x in v]) == 0
    assert [x.value for x in v] == [16, 16, 16, 1, 1]
    # no entry for bucket 4: the fixed choice for dense batches
    assert lib.rdseg_batched_lookup(arr, len(shapes), 0.9, *[ctypes.byref(x) for x in v]) == 0
    assert [x.value for x in v[:3]] == [64, 64, 8] and v[4].value == 0
    assert lib.rdseg_batched_lookup(arr, len(shapes), -0.1, *[ctypes.byref(x) for x in v]) == 1
    with pytest.raises(Exception):
        rdseg.tune_cache_import(json.dumps({"version": 1, "entries": [dict(entries[0], batched=2)]}))
    rdseg.tune_cache_clear()


def test_batched_autotune_validation(lib):
    arr = _fake_batch([(64, 64)])
    v = [ctypes.c_int32(0) for _ in range(4)]
    args = lambda probe, form, ws_bytes: (arr, 1, 0.1, 0.125, probe, 0, 0, 0, form,
                                          ctypes.c_void_p(8), ws_bytes, None,
                                          *[ctypes.byref(x) for x in v])
    assert lib.rdseg_autotune_batched(*args(0, 0, 1 << 40)) == 1    # probe_iters < 1
    assert lib.rdseg_autotune_batched(*args(10, 3, 1 << 40)) == 1   # form out of range
    assert lib.rdseg_autotune_batched(*args(10, 0, 16)) == 3        # workspace too small


def test_adjoint_form_validation(lib):
    """The reverse sweep's forms: the compiled (tile, steps) pairs are accepted
    (0, 0 restores the default), others are rejected with RDSEG_ERR_ARG."""
    try:
        for tile, steps in ((32, 1), (16, 2), (16, 4), (32, 2), (32, 4), (0, 0), (16, 0)):
            assert lib.rdseg_set_adjoint_form(tile, steps) == 0, (tile, steps)
        for tile, steps in ((64, 2), (32, 3), (16, 1), (8, 2), (-1, 2), (32, 9)):
            assert lib.rdseg_set_adjoint_form(tile, steps) == 1, (tile, steps)
    finally:
        assert lib.rdseg_set_adjoint_form(0, 0) == 0
