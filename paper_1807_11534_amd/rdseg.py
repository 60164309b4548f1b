"""PyTorch-facing binding of the HIP library (argument marshalling only).

torch provides device memory and the current HIP stream; every computation
runs in librdseg.so.  All image tensors are float32 CUDA (HIP) tensors with
unit stride along x; the row pitch is taken from the tensor's stride.
"""
import ctypes
import math

import torch

from . import _lib
from ._lib import Fit, Image, Params, Shape, check

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
           tile_h=0, ckpt_every=0):
    return Params(float(lam), float(theta), float(tau), float(delta), int(iters),
                  int(iters_per_launch), int(tile_w), int(tile_h), int(ckpt_every))


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


def solve(f, lam, theta=THETA, tau=TAU, delta=math.inf, iters=100, u0=None, p0=None,
          tile=None, iters_per_launch=0, ckpt_every=0, out=None, ws=None):
    """Restricted-domain dual iteration (Sec. 2.1 restricted as in Sec. 3).

    tile: (tile_w, tile_h) or None (autotuned).  Returns (u, v, p) with p of
    shape [2][H][W]; with ckpt_every > 0 returns (u, v, p, tape)."""
    lib = _lib.load()
    s = shape_of(f)
    tw, th = (0, 0) if tile is None else tile
    prm = params(lam, theta, tau, delta, iters, iters_per_launch, tw, th, ckpt_every)
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


def autotune(f, lam, theta=THETA, tau=TAU, delta=math.inf, probe_iters=16):
    """Time every compiled configuration on this problem; cache and return the best."""
    lib = _lib.load()
    s = shape_of(f)
    prm = params(lam, theta, tau, delta, probe_iters)
    u, v, p = _empty_like_grid(f), _empty_like_grid(f), _empty_like_grid(f, 2)
    ws = workspace(s, prm)
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib.rdseg_autotune(_vp(f), s, ctypes.byref(prm), int(probe_iters), _vp(u), _vp(v),
                             _vp(p), _vp(ws), ws.numel(), _stream(), ctypes.byref(a),
                             ctypes.byref(b), ctypes.byref(c)))
    return (a.value, b.value), c.value


def timing_enable(on=True):
    check(_lib.load().rdseg_timing_enable(1 if on else 0))


def timing_read():
    """(kernel_ms, launches, algorithmic_bytes, pixel_updates) since the last read."""
    ms, n, b, upd = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
    check(_lib.load().rdseg_timing_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b),
                                        ctypes.byref(upd)))
    return ms.value, n.value, b.value, upd.value
