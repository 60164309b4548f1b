"""FP64 CPU oracle for the restricted-domain dual segmentation method.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the HIP path.  The arithmetic lives in ``rdseg_oracle.c`` (plain C,
FP64, single thread); this module only marshals numpy arrays through ctypes.

Parity status of each function (pins live in ``tests/test_oracle_*.py``):

* ``active_set``  -- pinned (brute force on tiny grids, closed forms delta=inf / delta<=0).
* ``grad``/``div`` -- pinned (adjointness <grad u, p> = -<u, div p>; hand-worked 2x3 case).
* ``solve``       -- pinned (duality-gap certificate of the restricted energy, a brute-force
  dense projected primal-dual solve of that energy on 8x8 inputs, closed forms, symmetries,
  resume, invariants, monotone dual objective, independent matrix formulation).

``tests/test_oracle_mutants.py`` plants plausible mistakes (signs, indices, boundaries,
dropped terms, transposed operands, order) into copies of the C source and checks that
the pins above catch every one.
* ``dual_steps``  -- pinned (monotone dual objective, fixed point of the ROF dual).
* ``reverse``/``tangent`` -- pinned (dot-product identity, central finite differences).
* ``fit_term``/``fit_vjp`` -- pinned (hand-worked values, finite differences).
* ``count_needed`` -- pinned (exact rational ceiling via ``fractions``).
* ``band_threshold`` -- pinned (brute force over every candidate threshold on tiny
  inputs; exact fraction and minimality on larger ones; q = 0 / 1, ties, NaN, inf).
* ``solve_until`` -- pinned (diffs re-measured from two fixed-count solves; stop
  index; tolerance 0 / inf; empty domain stops at the first check).
* ``metrics``     -- pinned (hand-worked 2x3 case, identity, disjoint labels, symmetry).
* ``solve_pd``    -- pinned (duality gap of the restricted eq. CR problem closes; weak
  duality at every iterate; hand-derived two-pixel minimisers; mid-trajectory iterates
  of a dense-matrix formulation of the published algorithm).
* ``grad3``/``div3`` -- pinned (adjointness, hand-worked 2x2x2 case).
* ``solve3``      -- pinned (a volume of identical slices equals the pinned 2-D solve on
  each slice bit for bit; axis permutations; D = 1).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIBRARY selects another build of the same C source (the sanitizer build)
_LIB_PATH = os.environ.get("ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    _lib = _bind(_LIB_PATH)
    return _lib


def _bind(path):
    """Load a build of rdseg_oracle.c and declare its signatures (the tests
    also bind deliberately broken builds to check that the pins catch them)."""
    lib = ctypes.CDLL(path)
    c_int, c_double, c_size = ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.orc_active_set.argtypes = [_fp, c_int, c_int, c_double, _i32p, _u64p, _i32p,
                                   _i32p, _i32p, _i64p]
    lib.orc_grad.argtypes = [_dp, c_int, c_int, _dp, _dp]
    lib.orc_grad.restype = None
    lib.orc_div.argtypes = [_dp, _dp, c_int, c_int, _dp]
    lib.orc_div.restype = None
    lib.orc_solve.argtypes = [_fp, c_int, c_int, c_double, c_double, c_double, c_double,
                              c_int, c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_dual_steps.argtypes = [_fp, c_int, c_int, c_double, c_double, c_double, _dp,
                                   c_int, _dp, _dp]
    lib.orc_reverse.argtypes = [_fp, c_int, c_int, c_double, c_double, c_double, c_double,
                                c_int, _dp, _dp, _dp, _dp]
    lib.orc_tangent.argtypes = [_fp, c_int, c_int, c_double, c_double, c_double, c_double,
                                c_int, _dp, c_double, _dp, _dp]
    lib.orc_fit_term.argtypes = [_fp, _fp, c_size, c_double, c_double, c_double, _dp]
    lib.orc_fit_term.restype = None
    lib.orc_fit_vjp.argtypes = [_fp, _fp, c_size, c_double, c_double, _dp, _dp, _dp, _dp]
    lib.orc_fit_vjp.restype = None
    lib.orc_count_needed.argtypes = [c_double, ctypes.c_int64]
    lib.orc_count_needed.restype = ctypes.c_int64
    lib.orc_band_threshold.argtypes = [_fp, c_int, c_int, c_double, _dp]
    lib.orc_solve_until.argtypes = [_fp, c_int, c_int, c_double, c_double, c_double, c_double,
                                    c_int, c_double, c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                    ctypes.POINTER(c_int), _dp, c_int]
    lib.orc_metrics.argtypes = [_dp, _dp, c_size, c_double, _i64p, _i64p, _dp]
    lib.orc_metrics.restype = None
    lib.orc_solve_pd.argtypes = [_fp, c_int, c_int, c_double, c_double, c_double, c_double,
                                 c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_grad3.argtypes = [_dp, c_int, c_int, c_int, _dp, _dp, _dp]
    lib.orc_grad3.restype = None
    lib.orc_div3.argtypes = [_dp, _dp, _dp, c_int, c_int, c_int, _dp]
    lib.orc_div3.restype = None
    lib.orc_solve3.argtypes = [_fp, c_int, c_int, c_int, c_double, c_double, c_double, c_double,
                               c_int, c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    return lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"oracle {name} failed with code {rc}")


def active_set(f, delta):
    """Restricted domain |f| < delta as 8x8 tiles and as an ascending pixel list.

    Returns dict(tile_ids int32[n], masks uint64[n], slot_map int32[TH*TW],
    pixels int32[m]).  Paper: Sec. 3 (Fg/Bg/RD thresholding of the fitting term).
    """
    lib = _load()
    f = _f32(f)
    H, W = f.shape
    TH, TW = (H + 7) // 8, (W + 7) // 8
    nt_cap = TH * TW
    tile_ids = np.zeros(nt_cap, np.int32)
    masks = np.zeros(nt_cap, np.uint64)
    slot = np.zeros(nt_cap, np.int32)
    pix = np.zeros(H * W, np.int32)
    nt = ctypes.c_int32(0)
    npx = ctypes.c_int64(0)
    _check(lib.orc_active_set(_ptr(f, _fp), H, W, float(delta), _ptr(tile_ids, _i32p),
                              _ptr(masks, _u64p), _ptr(slot, _i32p), ctypes.byref(nt),
                              _ptr(pix, _i32p), ctypes.byref(npx)), "active_set")
    return dict(tile_ids=tile_ids[:nt.value].copy(), masks=masks[:nt.value].copy(),
                slot_map=slot, pixels=pix[:npx.value].copy())


def grad(u):
    """Forward-difference gradient of Chambolle (2004), zero on the last column/row."""
    lib = _load()
    u = _f64(u)
    H, W = u.shape
    gx = np.empty_like(u)
    gy = np.empty_like(u)
    lib.orc_grad(_ptr(u, _dp), H, W, _ptr(gx, _dp), _ptr(gy, _dp))
    return gx, gy


def div(px, py):
    """Divergence with div = -grad^T (Chambolle 2004)."""
    lib = _load()
    px, py = _f64(px), _f64(py)
    H, W = px.shape
    d = np.empty_like(px)
    lib.orc_div(_ptr(px, _dp), _ptr(py, _dp), H, W, _ptr(d, _dp))
    return d


def solve(f, lam, theta, tau, delta, iters, inner=1, u0=None, p0=None):
    """Restricted alternating dual iteration (Sec. 2.1 restricted as in Sec. 3).

    f: float32 [H][W] (held exactly in FP64).  u0: [H][W] or None (H(-f)).
    p0: [2][H][W] or None (zero).  Returns (u, v, p) in FP64, p as [2][H][W].
    """
    lib = _load()
    f = _f32(f)
    H, W = f.shape
    u = np.empty((H, W))
    v = np.empty((H, W))
    px = np.empty((H, W))
    py = np.empty((H, W))
    u0c = None if u0 is None else _f64(u0)
    p0x = None if p0 is None else _f64(p0[0])
    p0y = None if p0 is None else _f64(p0[1])
    _check(lib.orc_solve(_ptr(f, _fp), H, W, float(lam), float(theta), float(tau),
                         float(delta), int(iters), int(inner), _ptr(u0c, _dp),
                         _ptr(p0x, _dp), _ptr(p0y, _dp), _ptr(u, _dp), _ptr(v, _dp),
                         _ptr(px, _dp), _ptr(py, _dp)), "solve")
    return u, v, np.stack([px, py])


def dual_steps(f, v, theta, tau, delta, n, p0=None):
    """`n` restricted Chambolle fixed-point steps for p with v held fixed."""
    lib = _load()
    f = _f32(f)
    H, W = f.shape
    v = _f64(v)
    px = np.zeros((H, W)) if p0 is None else _f64(p0[0]).copy()
    py = np.zeros((H, W)) if p0 is None else _f64(p0[1]).copy()
    _check(lib.orc_dual_steps(_ptr(f, _fp), H, W, float(theta), float(tau), float(delta),
                              _ptr(v, _dp), int(n), _ptr(px, _dp), _ptr(py, _dp)),
           "dual_steps")
    return np.stack([px, py])


def reverse(f, lam, theta, tau, delta, iters, ubar, vbar=None):
    """Reverse-mode derivative of the unrolled solve (default start).

    Returns (fbar [H][W], lambar).  RD and u0 = H(-f) are held fixed.
    """
    lib = _load()
    f = _f32(f)
    H, W = f.shape
    ub = _f64(ubar)
    vb = None if vbar is None else _f64(vbar)
    fbar = np.empty((H, W))
    lb = ctypes.c_double(0.0)
    _check(lib.orc_reverse(_ptr(f, _fp), H, W, float(lam), float(theta), float(tau),
                           float(delta), int(iters), _ptr(ub, _dp), _ptr(vb, _dp),
                           _ptr(fbar, _dp), ctypes.byref(lb)), "reverse")
    return fbar, lb.value


def tangent(f, lam, theta, tau, delta, iters, df, dlam):
    """Forward-mode derivative of the final (u, v) along (df, dlam)."""
    lib = _load()
    f = _f32(f)
    H, W = f.shape
    dfc = _f64(df)
    du = np.empty((H, W))
    dv = np.empty((H, W))
    _check(lib.orc_tangent(_ptr(f, _fp), H, W, float(lam), float(theta), float(tau),
                           float(delta), int(iters), _ptr(dfc, _dp), float(dlam),
                           _ptr(du, _dp), _ptr(dv, _dp)), "tangent")
    return du, dv


def fit_term(z, c1, c2, gamma=0.0, P=None):
    """Fitting term of eq. CV (P None) or eq. DS, in FP64."""
    lib = _load()
    z = _f32(z)
    Pc = None if P is None else _f32(P)
    out = np.empty(z.shape)
    lib.orc_fit_term(_ptr(z, _fp), _ptr(Pc, _fp), z.size, float(c1), float(c2),
                     float(gamma), _ptr(out, _dp))
    return out


def fit_vjp(z, c1, c2, fbar, P=None):
    """(c1bar, c2bar, gammabar) = fbar . d f / d(c1, c2, gamma)."""
    lib = _load()
    z = _f32(z)
    Pc = None if P is None else _f32(P)
    fb = _f64(fbar)
    a, b, g = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib.orc_fit_vjp(_ptr(z, _fp), _ptr(Pc, _fp), z.size, float(c1), float(c2),
                    _ptr(fb, _dp), ctypes.byref(a), ctypes.byref(b), ctypes.byref(g))
    return a.value, b.value, g.value


def count_needed(q, n):
    """ceil(q n), exact: the number of RD nodes a fraction q of n asks for."""
    return int(_load().orc_count_needed(float(q), int(n)))


def band_threshold(f, q):
    """q-hat (Sec. 3): the smallest double with #{|f| < q-hat} >= q N."""
    lib = _load()
    f = _f32(f)
    H, W = f.shape
    out = ctypes.c_double()
    _check(lib.orc_band_threshold(_ptr(f, _fp), H, W, float(q), ctypes.byref(out)),
           "band_threshold")
    return out.value


def solve_until(f, lam, theta, tau, delta, max_iters, tol, check_every=1, u0=None, p0=None,
                inner=1):
    """Solve with the stopping rule of Sec. 4 evaluated every `check_every`
    iterations.  Returns (u, v, p, iterations run, measured values), p as
    [2][H][W]."""
    lib = _load()
    f = _f32(f)
    H, W = f.shape
    u = np.empty((H, W))
    v = np.empty((H, W))
    px = np.empty((H, W))
    py = np.empty((H, W))
    u0c = None if u0 is None else _f64(u0)
    p0x = None if p0 is None else _f64(p0[0])
    p0y = None if p0 is None else _f64(p0[1])
    diffs = np.full(max(1, max_iters // check_every), np.nan)
    done = ctypes.c_int()
    _check(lib.orc_solve_until(_ptr(f, _fp), H, W, float(lam), float(theta), float(tau),
                               float(delta), int(max_iters), float(tol), int(check_every),
                               _ptr(u0c, _dp), _ptr(p0x, _dp), _ptr(p0y, _dp),
                               _ptr(u, _dp), _ptr(v, _dp), _ptr(px, _dp), _ptr(py, _dp),
                               ctypes.byref(done), _ptr(diffs, _dp), int(inner)), "solve_until")
    n_checks = done.value // check_every
    return u, v, np.stack([px, py]), done.value, diffs[:n_checks]


def metrics(u, u_gt, eps=0.5):
    """Sec. 4 measures: (E1, E2, N(GT and Omega), N(GT or Omega))."""
    lib = _load()
    a = _f64(u)
    b = _f64(u_gt)
    assert a.shape == b.shape
    ni, nu, e2 = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    lib.orc_metrics(_ptr(a, _dp), _ptr(b, _dp), a.size, float(eps), ctypes.byref(ni),
                    ctypes.byref(nu), ctypes.byref(e2))
    e1 = 1.0 if nu.value == 0 else ni.value / nu.value
    return e1, e2.value, ni.value, nu.value


def grad3(u):
    """Forward-difference gradient of a volume [D][H][W]."""
    lib = _load()
    u = _f64(u)
    D, H, W = u.shape
    g = [np.empty_like(u) for _ in range(3)]
    lib.orc_grad3(_ptr(u, _dp), D, H, W, *[_ptr(a, _dp) for a in g])
    return tuple(g)


def div3(px, py, pz):
    """Divergence of a volume field, div = -grad^T."""
    lib = _load()
    px, py, pz = _f64(px), _f64(py), _f64(pz)
    D, H, W = px.shape
    d = np.empty_like(px)
    lib.orc_div3(_ptr(px, _dp), _ptr(py, _dp), _ptr(pz, _dp), D, H, W, _ptr(d, _dp))
    return d


def solve3(f, lam, theta, tau, delta, iters, inner=1, u0=None, p0=None):
    """Restricted iteration on a volume f [D][H][W]; returns (u, v, p) with p
    as [3][D][H][W]."""
    lib = _load()
    f = _f32(f)
    D, H, W = f.shape
    u, v = np.empty((D, H, W)), np.empty((D, H, W))
    p = np.empty((3, D, H, W))
    u0c = None if u0 is None else _f64(u0)
    p0c = None if p0 is None else [_f64(a) for a in p0]
    _check(lib.orc_solve3(_ptr(f, _fp), D, H, W, float(lam), float(theta), float(tau),
                          float(delta), int(iters), int(inner), _ptr(u0c, _dp),
                          *(([None] * 3) if p0c is None else [_ptr(a, _dp) for a in p0c]),
                          _ptr(u, _dp), _ptr(v, _dp), _ptr(p[0], _dp), _ptr(p[1], _dp),
                          _ptr(p[2], _dp)), "solve3")
    return u, v, p


def solve_pd(f, lam, tau, sigma, delta, iters, u0=None, p0=None):
    """Restricted primal-dual (Chambolle-Pock) iteration for eq. CR; returns
    (u, p) with p as [2][H][W]."""
    lib = _load()
    f = _f32(f)
    H, W = f.shape
    u = np.empty((H, W))
    px, py = np.empty((H, W)), np.empty((H, W))
    u0c = None if u0 is None else _f64(u0)
    p0x = None if p0 is None else _f64(p0[0])
    p0y = None if p0 is None else _f64(p0[1])
    _check(lib.orc_solve_pd(_ptr(f, _fp), H, W, float(lam), float(tau), float(sigma),
                            float(delta), int(iters), _ptr(u0c, _dp), _ptr(p0x, _dp),
                            _ptr(p0y, _dp), _ptr(u, _dp), _ptr(px, _dp), _ptr(py, _dp)),
           "solve_pd")
    return u, np.stack([px, py])
