"""PyTorch-facing binding of the HIP library (argument marshalling only).

torch provides device memory and the current HIP stream; every computation
runs in librdseg.so.  All image tensors are float32 CUDA (HIP) tensors with
unit stride along x; the row pitch is taken from the tensor's stride.
"""
import ctypes
import math

import torch

from . import _lib
from ._lib import Fit, Image, Params, PdParams, Shape, Shape3, check

THETA = 0.1
TAU = 0.125


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_plane(t, name, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 tensor on the GPU")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit stride along x")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def shape_of(f):
    _check_plane(f, "f")
    H, W = f.shape
    return Shape(H, W, f.stride(0))


def params(lam, theta=THETA, tau=TAU, delta=math.inf, iters=0, iters_per_launch=0, tile_w=0,
           tile_h=0, ckpt_every=0, inner=1, components=0, resident=0):
    return Params(float(lam), float(theta), float(tau), float(delta), int(iters),
                  int(iters_per_launch), int(tile_w), int(tile_h), int(ckpt_every), int(inner),
                  int(components), int(resident))


def workspace(s, prm=None):
    n = _lib.load().rdseg_workspace_size(ctypes.byref(s), None if prm is None else ctypes.byref(prm))
    if n == 0:
        raise ValueError("invalid shape")
    return torch.empty(n, dtype=torch.uint8, device="cuda")


def _empty_like_grid(f, planes=None):
    H, W = f.shape
    ld = f.stride(0)
    if planes is None:
        return torch.empty((H, ld), dtype=torch.float32, device=f.device)[:, :W]
    return torch.empty((planes, H, ld), dtype=torch.float32, device=f.device)[:, :, :W]


def active_set(f, delta, pixels=True):
    """Restricted domain |f| < delta as 8x8 tiles (+ ascending pixel list).

    Returns dict of tensors trimmed to their counts (synchronises)."""
    lib = _lib.load()
    s = shape_of(f)
    TH, TW = (s.H + 7) // 8, (s.W + 7) // 8
    dev = f.device
    ids = torch.empty(TH * TW, dtype=torch.int32, device=dev)
    masks = torch.empty(TH * TW, dtype=torch.int64, device=dev)
    slot = torch.empty(TH * TW, dtype=torch.int32, device=dev)
    nt = torch.zeros(1, dtype=torch.int32, device=dev)
    pix = torch.empty(s.H * s.W, dtype=torch.int32, device=dev) if pixels else None
    npx = torch.zeros(1, dtype=torch.int64, device=dev) if pixels else None
    ws = workspace(s)
    check(lib.rdseg_active_set(_vp(f), s, float(delta), _vp(ids), _vp(masks), _vp(slot), _vp(nt),
                               _vp(pix), _vp(npx), _vp(ws), ws.numel(), _stream()))
    n = int(nt.item())
    out = dict(tile_ids=ids[:n], masks=masks[:n], slot_map=slot)
    if pixels:
        out["pixels"] = pix[: int(npx.item())]
    return out


def band_threshold(f, q, out=None, ws=None):
    """q-hat of Sec. 3 for a target fraction q of nodes in the restricted
    domain, as a device float64 scalar tensor (no synchronisation)."""
    lib = _lib.load()
    s = shape_of(f)
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=f.device)
    if ws is None:
        ws = torch.empty(lib.rdseg_band_workspace_size(), dtype=torch.uint8, device=f.device)
    check(lib.rdseg_band_threshold(_vp(f), s, float(q), _vp(out), _vp(ws), ws.numel(),
                                   _stream()))
    return out


def delta_for_fraction(f, q):
    """q-hat as a Python float (synchronises once)."""
    return float(band_threshold(f, q).item())


def solve(f, lam, theta=THETA, tau=TAU, delta=math.inf, iters=100, u0=None, p0=None,
          tile=None, iters_per_launch=0, ckpt_every=0, out=None, ws=None, inner=1,
          components=0, resident=0):
    """Restricted-domain dual iteration (Sec. 2.1 restricted as in Sec. 3).

    tile: (tile_w, tile_h) or None (autotuned); inner: dual steps per outer
    iteration; components: small-component path, 1 on, 2 off, 0 the library's
    choice (see autotune); resident: barrier between blocks of iterations, 1
    on-chip exchange where the tiles fit, 2 separate launches, 0 the library's
    choice.  Returns (u, v, p) with p of shape [2][H][W]; with ckpt_every > 0
    returns (u, v, p, tape)."""
    lib = _lib.load()
    s = shape_of(f)
    tw, th = (0, 0) if tile is None else tile
    prm = params(lam, theta, tau, delta, iters, iters_per_launch, tw, th, ckpt_every, inner,
                 components, resident)
    if out is None:
        u, v, p = _empty_like_grid(f), _empty_like_grid(f), _empty_like_grid(f, 2)
    else:
        u, v, p = out
    if p.stride(0) != s.H * s.ld or p.stride(1) != s.ld:
        raise ValueError("p must be [2][H][ld] with the pitch of f")
    tape = None
    if ckpt_every > 0:
        nbytes = lib.rdseg_tape_size(ctypes.byref(s), ctypes.byref(prm))
        tape = torch.empty(max(nbytes // 4, 1), dtype=torch.float32, device=f.device)
    if ws is None:
        ws = workspace(s, prm)
    check(lib.rdseg_solve(_vp(f), s, ctypes.byref(prm), _vp(u0), _vp(p0), _vp(u), _vp(v), _vp(p),
                          _vp(tape), _vp(ws), ws.numel(), _stream()))
    if ckpt_every > 0:
        return u, v, p, tape
    return u, v, p


def solve_status(f, ws):
    """Status of the last solve of f's shape that used workspace ws
    (synchronises the current stream): 0, or 6 (RDSEG_ERR_TIMEOUT) when a
    resident solve's bounded wait expired and its affected tiles hold NaN."""
    lib = _lib.load()
    s = shape_of(f)
    st = lib.rdseg_solve_status(ctypes.byref(s), _vp(ws), ws.numel(), _stream())
    if st not in (_lib.RDSEG_OK, _lib.RDSEG_ERR_TIMEOUT):
        check(st)
    return st


def set_resident_wait(ticks):
    """Bound of each resident-form wait in 100 MHz wall-clock ticks (0: the
    default of one second; < 0: every wait gives up at once, for tests)."""
    check(_lib.load().rdseg_set_resident_wait(int(ticks)))


def solve_until(f, lam, theta=THETA, tau=TAU, delta=math.inf, max_iters=1000, tol=1e-2,
                check_every=1, u0=None, p0=None, tile=None, iters_per_launch=0, out=None,
                ws=None, poll=True, inner=1):
    """Solve with the stopping rule of Sec. 4 (maximum-norm change of u and v
    at most tol, checked every `check_every` iterations, decided on the device).
    poll: read the checks back in growing chunks and stop enqueuing soon after
    the stop (synchronises); False enqueues all max_iters iterations.

    Returns (u, v, p, iters_done, diffs): iters_done a device int32 scalar,
    diffs the device float32 changes at each check (zeros after the stop)."""
    lib = _lib.load()
    s = shape_of(f)
    tw, th = (0, 0) if tile is None else tile
    prm = params(lam, theta, tau, delta, max_iters, iters_per_launch, tw, th, 0, inner)
    if out is None:
        u, v, p = _empty_like_grid(f), _empty_like_grid(f), _empty_like_grid(f, 2)
    else:
        u, v, p = out
    if p.stride(0) != s.H * s.ld or p.stride(1) != s.ld:
        raise ValueError("p must be [2][H][ld] with the pitch of f")
    n_checks = max_iters // check_every if max_iters > 0 and check_every > 0 else 0
    diffs = torch.zeros(max(n_checks, 1), dtype=torch.float32, device=f.device)
    done = torch.zeros((), dtype=torch.int32, device=f.device)
    if ws is None:
        ws = workspace(s, prm)
    check(lib.rdseg_solve_until(_vp(f), s, ctypes.byref(prm), float(tol), int(check_every),
                                1 if poll else 0, _vp(u0), _vp(p0), _vp(u), _vp(v), _vp(p), _vp(done), _vp(diffs),
                                _vp(ws), ws.numel(), _stream()))
    return u, v, p, done, diffs[:n_checks]


def metrics(u, u_ref, eps=0.5, out=None, ws=None):
    """Sec. 4 measures on the device: tensor [N(GT and Omega), N(GT or Omega),
    E2] (float64, no synchronisation); E1 = out[0] / out[1]."""
    lib = _lib.load()
    s = shape_of(u)
    if shape_of(u_ref).H != s.H or shape_of(u_ref).W != s.W or u_ref.stride(0) != s.ld:
        raise ValueError("u_ref must have the shape and pitch of u")
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=u.device)
    if ws is None:
        ws = torch.empty(lib.rdseg_metrics_workspace_size(), dtype=torch.uint8, device=u.device)
    check(lib.rdseg_metrics(_vp(u), _vp(u_ref), s, float(eps), _vp(out), _vp(ws), ws.numel(),
                            _stream()))
    return out


def e1_e2(u, u_ref, eps=0.5):
    """(E1, E2) of Sec. 4 as Python floats (synchronises)."""
    a, b, e2 = metrics(u, u_ref, eps).tolist()
    return (1.0 if b == 0 else a / b), e2


PD_STEP = 1.0 / math.sqrt(8.0)   # tau = sigma with tau * sigma * |grad|^2 <= 1


def solve_pd(f, lam, delta=math.inf, iters=500, tau=PD_STEP, sigma=PD_STEP, u0=None, p0=None,
             tile=None, iters_per_launch=0, out=None, ws=None):
    """The restricted primal-dual (Chambolle-Pock) iteration for eq. CR.
    Returns (u, p) with p of shape [2][H][W]."""
    lib = _lib.load()
    s = shape_of(f)
    tw, th = (0, 0) if tile is None else tile
    prm = PdParams(float(lam), float(tau), float(sigma), float(delta), int(iters),
                   int(iters_per_launch), int(tw), int(th))
    if out is None:
        u, p = _empty_like_grid(f), _empty_like_grid(f, 2)
    else:
        u, p = out
    if p.stride(0) != s.H * s.ld or p.stride(1) != s.ld:
        raise ValueError("p must be [2][H][ld] with the pitch of f")
    if ws is None:
        n = lib.rdseg_pd_workspace_size(ctypes.byref(s))
        if n == 0:
            raise ValueError("invalid shape")
        ws = torch.empty(n, dtype=torch.uint8, device=f.device)
    check(lib.rdseg_solve_pd(_vp(f), s, ctypes.byref(prm), _vp(u0), _vp(p0), _vp(u), _vp(p),
                             _vp(ws), ws.numel(), _stream()))
    return u, p


def shape3_of(f):
    if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dtype != torch.float32:
        raise TypeError("f must be a float32 tensor on the GPU")
    if f.dim() != 3 or f.stride(2) != 1:
        raise ValueError("a volume must be 3-D [D][H][W] with unit stride along x")
    D, H, W = f.shape
    return Shape3(D, H, W, f.stride(1), f.stride(0))


def _empty_like_volume(f, planes=None):
    D, H, W = f.shape
    ld, lds = f.stride(1), f.stride(0)
    n = D * lds if planes is None else planes * D * lds
    buf = torch.empty(n, dtype=torch.float32, device=f.device)
    if planes is None:
        return buf.as_strided((D, H, W), (lds, ld, 1))
    return buf.as_strided((planes, D, H, W), (D * lds, lds, ld, 1))


def solve3d(f, lam, theta=THETA, tau=1.0 / 12.0, delta=math.inf, iters=100, inner=1, u0=None,
            p0=None, out=None, ws=None):
    """The restricted iteration on a volume f [D][H][W] (7-point stencil).
    Returns (u, v, p) with p of shape [3][D][H][W] (x, y, z components)."""
    lib = _lib.load()
    s = shape3_of(f)
    prm = params(lam, theta, tau, delta, iters, 0, 0, 0, 0, inner)
    if out is None:
        u, v, p = _empty_like_volume(f), _empty_like_volume(f), _empty_like_volume(f, 3)
    else:
        u, v, p = out
    if ws is None:
        n = lib.rdseg_workspace_size3(ctypes.byref(s))
        if n == 0:
            raise ValueError("invalid volume shape")
        ws = torch.empty(n, dtype=torch.uint8, device=f.device)
    check(lib.rdseg_solve3d(_vp(f), s, ctypes.byref(prm), _vp(u0), _vp(p0), _vp(u), _vp(v),
                            _vp(p), _vp(ws), ws.numel(), _stream()))
    return u, v, p


class BatchedSolver:
    """Many independent images solved over one global tile queue.

    graph=True captures the whole sequence (init, compaction, every iteration
    launch) into a hipGraph on the first run and replays it afterwards; only
    the contents of the f tensors may change between runs."""

    def __init__(self, fs, lams, deltas, theta=THETA, tau=TAU, iters=100, tile=(32, 32),
                 iters_per_launch=4, graph=True):
        """tile=None with iters_per_launch=0 leaves the configuration (and the
        form of the iterations) to the library: the tuning cache's entry for
        the batch (see autotune), else a fixed choice by active fraction."""
        self.lib = _lib.load()
        n = len(fs)
        if not (len(lams) == len(deltas) == n and n > 0):
            raise ValueError("fs, lams and deltas must have the same non-zero length")
        self.fs = list(fs)
        self.out = []
        arr = (Image * n)()
        for i, f in enumerate(self.fs):
            s = shape_of(f)
            u, v, p = _empty_like_grid(f), _empty_like_grid(f), _empty_like_grid(f, 2)
            self.out.append((u, v, p))
            arr[i] = Image(f.data_ptr(), u.data_ptr(), v.data_ptr(), p.data_ptr(), s,
                           float(lams[i]), float(deltas[i]))
        self.imgs = arr
        self.n = n
        self.theta, self.tau, self.iters = float(theta), float(tau), int(iters)
        self.tile, self.ipl = (tile if tile is not None else (0, 0)), int(iters_per_launch)
        self.graph = graph
        self.plan = ctypes.c_void_p(None)
        self.ws = None
        if not graph:
            nbytes = self.lib.rdseg_batched_workspace_size(arr, n, self.tile[0], self.tile[1])
            if nbytes == 0:
                raise ValueError("invalid batch")
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.fs[0].device)

    def run(self):
        plan = ctypes.byref(self.plan) if self.graph else None
        ws = self.ws
        check(self.lib.rdseg_solve_batched(self.imgs, self.n, self.theta, self.tau, self.iters,
                                           self.ipl, self.tile[0], self.tile[1], plan, _vp(ws),
                                           0 if ws is None else ws.numel(), _stream()))
        return self.out

    def autotune(self, probe_iters=None, tile=None, iters_per_launch=0, form=0):
        """Time every configuration and both forms of the iterations on this
        batch (rdseg_autotune_batched; the outputs are overwritten) and return
        Tuned ((tile_w, tile_h), iters_per_launch) with `.form`; an
        unrestricted search is stored in the tuning cache, which a solve that
        leaves the choice to the library reads."""
        nbytes = self.lib.rdseg_batched_workspace_size(self.imgs, self.n, 0, 0)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.fs[0].device)
        tw, th = (0, 0) if tile is None else tile
        v = [ctypes.c_int32(0) for _ in range(4)]
        check(self.lib.rdseg_autotune_batched(
            self.imgs, self.n, self.theta, self.tau, int(probe_iters or self.iters), int(tw),
            int(th), int(iters_per_launch), int(form), _vp(ws), ws.numel(), _stream(),
            *[ctypes.byref(x) for x in v]))
        t = Tuned((v[0].value, v[1].value), v[2].value, 2, v[3].value)
        t.form = v[3].value
        return t

    def lookup(self, q):
        """The configuration and form a library-chosen solve of this batch
        uses when its active fraction is q (host only)."""
        v = [ctypes.c_int32(0) for _ in range(5)]
        check(self.lib.rdseg_batched_lookup(self.imgs, self.n, float(q),
                                            *[ctypes.byref(x) for x in v]))
        t = Tuned((v[0].value, v[1].value), v[2].value, 2, v[3].value)
        t.form, t.cached = v[3].value, bool(v[4].value)
        return t

    def close(self):
        if self.plan.value:
            check(self.lib.rdseg_plan_destroy(self.plan))
            self.plan = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def as_grid_of(t, like):
    """t in the layout of the plane `like` (same shape, row pitch and unit
    stride along x): t itself when it already is, else a copy (any strides,
    expanded ones included)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError("a gradient must be a float32 tensor on the GPU")
    if tuple(t.shape) != tuple(like.shape):
        raise ValueError(f"gradient has shape {tuple(t.shape)}, expected {tuple(like.shape)}")
    if t.stride(1) == 1 and t.stride(0) == like.stride(0):
        return t
    out = _empty_like_grid(like)
    out.copy_(t)
    return out


def backward(f, lam, theta, tau, delta, iters, ckpt_every, tape, grad_u, grad_v=None,
             fit=None):
    """Reverse mode of the solve that wrote `tape` (default start).

    fit: None or (z, P or None, c1, c2, gamma) -- the f of the solve came from
    fit_forward with these values.  grad_u / grad_v are read with f's row
    pitch (copied into that layout when theirs differs).  Returns (grad_f,
    grad_lambda) and, with fit, (grad_c1, grad_c2, grad_gamma) as float64
    device scalars."""
    lib = _lib.load()
    s = shape_of(f)
    grad_u = as_grid_of(grad_u, f)
    if grad_v is not None:
        grad_v = as_grid_of(grad_v, f)
    if fit is not None:
        _check_plane(fit[0], "z", f.shape)
        if fit[0].stride(0) != f.stride(0) or (fit[1] is not None and
                                               fit[1].stride(0) != f.stride(0)):
            raise ValueError("z and P must have the row pitch of f")
    prm = params(lam, theta, tau, delta, iters, 0, 0, 0, ckpt_every)
    nbytes = lib.rdseg_backward_workspace_size(ctypes.byref(s), ctypes.byref(prm))
    if nbytes == 0:
        raise ValueError("invalid shape or ckpt_every")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=f.device)
    gf = _empty_like_grid(f)
    scal = torch.zeros(4, dtype=torch.float64, device=f.device)
    fitp = None
    if fit is not None:
        z, P, c1, c2, gamma = fit
        fitp = ctypes.byref(Fit(z.data_ptr(), None if P is None else P.data_ptr(), float(c1),
                                float(c2), float(gamma)))
    check(lib.rdseg_backward(_vp(f), s, ctypes.byref(prm), _vp(tape), _vp(grad_u), _vp(grad_v),
                             _vp(gf), ctypes.c_void_p(scal.data_ptr()), fitp,
                             ctypes.c_void_p(scal.data_ptr() + 8),
                             ctypes.c_void_p(scal.data_ptr() + 16),
                             ctypes.c_void_p(scal.data_ptr() + 24), _vp(ws), ws.numel(),
                             _stream()))
    if fit is None:
        return gf, scal[0]
    return gf, scal[0], scal[1], scal[2], scal[3]


def fit_forward(z, c1, c2, gamma=0.0, P=None):
    """Fitting term of eq. CV (P None) or eq. DS, evaluated on the GPU."""
    lib = _lib.load()
    s = shape_of(z)
    f = _empty_like_grid(z)
    fit = Fit(z.data_ptr(), None if P is None else P.data_ptr(), float(c1), float(c2),
              float(gamma))
    check(lib.rdseg_fit_forward(ctypes.byref(fit), s, _vp(f), _stream()))
    return f


def fit_backward(z, c1, c2, grad_f, P=None):
    """(dL/dc1, dL/dc2, dL/dgamma) from dL/df, as float64 device scalars.
    grad_f is read with z's row pitch (copied into that layout when its own
    differs)."""
    lib = _lib.load()
    s = shape_of(z)
    grad_f = as_grid_of(grad_f, z)
    if P is not None and P.stride(0) != z.stride(0):
        raise ValueError("P must have the row pitch of z")
    nbytes = lib.rdseg_reduce_workspace_size(ctypes.byref(s))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=z.device)
    out = torch.zeros(3, dtype=torch.float64, device=z.device)
    fit = Fit(z.data_ptr(), None if P is None else P.data_ptr(), float(c1), float(c2), 0.0)
    check(lib.rdseg_fit_backward(ctypes.byref(fit), s, _vp(grad_f),
                                 ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr() + 8),
                                 ctypes.c_void_p(out.data_ptr() + 16), _vp(ws), ws.numel(),
                                 _stream()))
    return out[0], out[1], out[2]


def configs():
    """Compiled (tile_w, tile_h, iters_per_launch, threads) configurations."""
    lib = _lib.load()
    out = []
    for i in range(lib.rdseg_config_count()):
        a, b, c, d = (ctypes.c_int32() for _ in range(4))
        check(lib.rdseg_config_get(i, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                   ctypes.byref(d)))
        out.append((a.value, b.value, c.value, d.value))
    return out


class Tuned(tuple):
    """((tile_w, tile_h), iters_per_launch) of an autotuned configuration; the
    small-component choice (1 on, 2 off) rides along as `.components` and the
    barrier kind (1 on-chip exchange, 2 separate launches) as `.resident`."""

    def __new__(cls, tile, ipl, components, resident=1):
        t = super().__new__(cls, (tile, ipl))
        t.components = components
        t.resident = resident
        return t


def autotune(f, lam, theta=THETA, tau=TAU, delta=math.inf, probe_iters=16, iters_per_launch=0,
             tile=None, components=0, resident=0):
    """Time every compiled configuration, with the small-component path on and
    off and both barrier kinds where the tiles fit on the chip, on this
    problem and return the best as Tuned ((tile_w, tile_h), iters_per_launch)
    with `.components` and `.resident`.  A nonzero iters_per_launch, tile,
    components or resident fixes that parameter and only matching candidates
    are timed; an unrestricted search is also cached for solves that leave
    the choice to the library."""
    lib = _lib.load()
    s = shape_of(f)
    tw, th = (0, 0) if tile is None else tile
    prm = params(lam, theta, tau, delta, probe_iters, iters_per_launch=iters_per_launch, tile_w=tw,
                 tile_h=th, components=components, resident=resident)
    u, v, p = _empty_like_grid(f), _empty_like_grid(f), _empty_like_grid(f, 2)
    ws = workspace(s, prm)
    a, b, c, k, r = (ctypes.c_int32() for _ in range(5))
    check(lib.rdseg_autotune(_vp(f), s, ctypes.byref(prm), int(probe_iters), _vp(u), _vp(v),
                             _vp(p), _vp(ws), ws.numel(), _stream(), ctypes.byref(a),
                             ctypes.byref(b), ctypes.byref(c), ctypes.byref(k), ctypes.byref(r)))
    return Tuned((a.value, b.value), c.value, k.value, r.value)


def timing_enable(on=True):
    check(_lib.load().rdseg_timing_enable(1 if on else 0))


def timing_read(config=-1):
    """(kernel_ms, launches, algorithmic_bytes, pixel_updates) of the recorded
    iteration-kernel launches of one configuration index (-1 = all)."""
    ms, n, b, upd = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
    check(_lib.load().rdseg_timing_read(int(config), ctypes.byref(ms), ctypes.byref(n),
                                        ctypes.byref(b), ctypes.byref(upd)))
    return ms.value, n.value, b.value, upd.value


def timing_read_form(config=-1, form=-1):
    """As timing_read, for one form of launch: 0 = separate launches of the
    blocked kernel, 1 = resident launches (one per solve), -1 = both."""
    ms, n, b, upd = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
    check(_lib.load().rdseg_timing_read_form(int(config), int(form), ctypes.byref(ms),
                                             ctypes.byref(n), ctypes.byref(b), ctypes.byref(upd)))
    return ms.value, n.value, b.value, upd.value


def set_resident(on=True):
    """Allow (default) or forbid the resident form of single-image solves."""
    check(_lib.load().rdseg_set_resident(1 if on else 0))


def set_batched_form(form):
    """Batched solves with a fixed configuration: 1 = every block of
    iterations in one persistent cooperative launch, 2 = one launch per block
    (default)."""
    check(_lib.load().rdseg_set_batched_form(int(form)))


def set_adjoint_form(tile=0, steps=0):
    """Form of the backward's reverse sweep: `steps` reverse iterations per
    launch on tile x tile macro tiles (0, 0 = the default, 32 and 2)."""
    check(_lib.load().rdseg_set_adjoint_form(int(tile), int(steps)))


def set_components(on=True):
    """Allow (default) or forbid the small-component path of single-image solves."""
    check(_lib.load().rdseg_set_components(1 if on else 0))


def tune_cache_export():
    """The autotuner's cache as JSON text (see rdseg_tune_cache_export)."""
    lib = _lib.load()
    n = ctypes.c_size_t(0)
    lib.rdseg_tune_cache_export(None, 0, ctypes.byref(n))   # asks for the size
    buf = ctypes.create_string_buffer(n.value)
    check(lib.rdseg_tune_cache_export(buf, n.value, ctypes.byref(n)))
    return buf.value.decode()


def tune_cache_import(text):
    """Merge JSON text of rdseg_tune_cache_export's form into the cache."""
    check(_lib.load().rdseg_tune_cache_import(text.encode()))


def tune_lookup(shape, q):
    """The configuration a library-chosen solve uses for an image of `shape`
    ((H, W) or a Shape) whose RD holds the fraction q of its pixels: Tuned
    ((tile_w, tile_h), iters_per_launch) with `.components` / `.resident`
    (0 = the library's default) and `.cached` (whether it came from the
    tuning cache)."""
    lib = _lib.load()
    s = shape if isinstance(shape, Shape) else Shape(int(shape[0]), int(shape[1]), int(shape[1]))
    v = [ctypes.c_int32(0) for _ in range(6)]
    check(lib.rdseg_tune_lookup(ctypes.byref(s), float(q), *[ctypes.byref(x) for x in v]))
    t = Tuned((v[0].value, v[1].value), v[2].value, v[3].value, v[4].value)
    t.cached = bool(v[5].value)
    return t


def tune_cache_clear():
    check(_lib.load().rdseg_tune_cache_clear())


def tune_cache_save(path):
    with open(path, "w") as fh:
        fh.write(tune_cache_export())


def tune_cache_load(path):
    with open(path) as fh:
        tune_cache_import(fh.read())


def timing_reset():
    check(_lib.load().rdseg_timing_reset())


def config_index(tile, iters_per_launch):
    for i, (tw, th, it, _) in enumerate(configs()):
        if (tw, th) == tuple(tile) and it == iters_per_launch:
            return i
    raise ValueError("configuration not compiled")
