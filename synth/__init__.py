"""Seeded synthetic inputs for the restricted-domain dual segmentation workloads.

This module is shared by the oracle side (tests) and the GPU side (tests,
benchmark).  It holds no arithmetic of the segmentation method itself: it only
draws images, masks and marker distances, and composes the fitting-term input
field f of Sec. 1 (eq. CV, eq. DS) once in FP64 before a single rounding to
FP32.  Every generator takes an explicit seed and uses numpy's PCG64.

The paper's own 128x128 test images (Examples 1-3) are not available; the
recipes below stand in for them with the sizes, intensity levels and noise
levels of the benchmark workloads:

* ``disc_rect_image``: background 0.2, a disc (radius 30 at (y, x) = (64, 40)
  on a 128x128 grid) and a rectangle (x in [80, 118), y in [20, 108)) at 0.8,
  geometry scaled by (H/128, W/128) for other sizes, plus N(0, sigma^2) noise;
  c1 = 0.8, c2 = 0.2.
* ``ellipses_image``: background U[0.1, 0.3]; `n` ellipses with centre
  U[0.15, 0.85] * S, semi-axes U[lo, hi] * S, angle U[0, pi), intensity
  U[0.6, 0.9], painted in order; noise sigma; c1 / c2 are the means of the noisy
  image over the ellipses / the rest.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

THETA = 0.1
TAU = 0.125


@dataclass
class Problem:
    """One segmentation input: f (float32 [H][W]) plus the data it came from."""
    f: np.ndarray
    z: np.ndarray                 # float32 image
    mask: np.ndarray              # bool, noise-free foreground
    c1: float
    c2: float
    gamma: float = 0.0
    P: Optional[np.ndarray] = None   # float32 distance term (eq. DS) or None
    lam: float = 5.0
    theta: float = THETA
    tau: float = TAU
    delta: float = float("inf")
    iters: int = 200
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.f.shape


def compose_f(z64, c1, c2, gamma=0.0, P64=None):
    """Fitting-term input of eq. CV / eq. DS, in FP64 (rounded by the caller)."""
    f = (z64 - c1) ** 2 - (z64 - c2) ** 2
    if P64 is not None:
        f = f + gamma * P64
    return f


def disc_rect_image(H, W, seed, sigma=0.05):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    sy, sx = H / 128.0, W / 128.0
    disc = ((x - 40 * sx) / (30 * sx)) ** 2 + ((y - 64 * sy) / (30 * sy)) ** 2 <= 1.0
    rect = (x >= 80 * sx) & (x < 118 * sx) & (y >= 20 * sy) & (y < 108 * sy)
    mask = disc | rect
    z = np.where(mask, 0.8, 0.2) + rng.normal(0.0, sigma, (H, W))
    return z, mask


def ellipses_image(S, n, semi_lo, semi_hi, sigma, seed):
    rng = np.random.default_rng(seed)
    bg = rng.uniform(0.1, 0.3)
    z = np.full((S, S), bg)
    mask = np.zeros((S, S), bool)
    y, x = np.mgrid[0:S, 0:S].astype(np.float64)
    for _ in range(n):
        cy, cx = rng.uniform(0.15, 0.85, 2) * S
        a, b = rng.uniform(semi_lo, semi_hi, 2) * S
        ang = rng.uniform(0.0, np.pi)
        ca, sa = np.cos(ang), np.sin(ang)
        # local window for speed
        r = int(np.ceil(max(a, b))) + 2
        y0, y1 = max(0, int(cy) - r), min(S, int(cy) + r + 1)
        x0, x1 = max(0, int(cx) - r), min(S, int(cx) + r + 1)
        yy, xx = y[y0:y1, x0:x1] - cy, x[y0:y1, x0:x1] - cx
        xr = ca * xx + sa * yy
        yr = -sa * xx + ca * yy
        inside = (xr / a) ** 2 + (yr / b) ** 2 <= 1.0
        val = rng.uniform(0.6, 0.9)
        z[y0:y1, x0:x1][inside] = val
        mask[y0:y1, x0:x1][inside] = True
    z = z + rng.normal(0.0, sigma, (S, S))
    return z, mask, rng


def _region_means(z, mask):
    c1 = float(z[mask].mean()) if mask.any() else 1.0
    c2 = float(z[~mask].mean()) if (~mask).any() else 0.0
    return c1, c2


def _finish(z64, mask, c1, c2, gamma=0.0, P64=None, **kw):
    f64 = compose_f(z64, c1, c2, gamma, P64)
    return Problem(f=f64.astype(np.float32), z=z64.astype(np.float32), mask=mask,
                   c1=c1, c2=c2, gamma=gamma,
                   P=None if P64 is None else P64.astype(np.float32), **kw)


def band_delta(f, frac):
    """delta = frac * max|f|, computed in FP64 from the FP32 field (inf stays inf)."""
    if not np.isfinite(frac):
        return float("inf")
    return float(frac) * float(np.abs(f.astype(np.float64)).max())


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def config1(seed=0, H=128, W=128):
    """Plain method on the disc + rectangle image; lambda 5, full domain, 200 iterations."""
    z, mask = disc_rect_image(H, W, seed)
    return _finish(z, mask, 0.8, 0.2, lam=5.0, delta=float("inf"), iters=200,
                   meta=dict(name="disc_rect", seed=seed))


C2_LAMBDAS = (1.0, 5.0, 20.0)
C2_FRACS = (float("inf"), 0.5, 0.2, 0.05)


def config2(lam_index=0, size=1024, iters=500):
    """Ellipse image for the restricted-domain sweep; one image per lambda (seeds 1..3)."""
    seed = 1 + lam_index
    z, mask, _ = ellipses_image(size, 6, 0.04, 0.15, 0.05, seed)
    c1, c2 = _region_means(z, mask)
    return _finish(z, mask, c1, c2, lam=C2_LAMBDAS[lam_index], iters=iters,
                   meta=dict(name="ellipses6", seed=seed))


def config3(size=4096, iters=1000, seed=7):
    """40 blobs, distance-selective term (gamma 2, 5 markers), lambda 10, delta 0.1 max|f|."""
    z, mask, rng = ellipses_image(size, 40, 0.01, 0.05, 0.08, seed)
    c1, c2 = _region_means(z, mask)
    fg = np.flatnonzero(mask.ravel())
    if fg.size == 0:
        fg = np.arange(size * size)
    mk = rng.choice(fg, 5, replace=False)
    my, mx = np.divmod(mk, size)
    y, x = np.mgrid[0:size, 0:size].astype(np.float64)
    dist = np.full((size, size), np.inf)
    for a, b in zip(my, mx):
        dist = np.minimum(dist, np.sqrt((y - a) ** 2 + (x - b) ** 2))
    P = dist / dist.max()
    prob = _finish(z, mask, c1, c2, gamma=2.0, P64=P, lam=10.0, iters=iters,
                   meta=dict(name="blobs40_ds", seed=seed, markers=list(zip(my.tolist(), mx.tolist()))))
    prob.delta = band_delta(prob.f, 0.1)
    return prob


def config4_image(i, lo=64, hi=1024, frac=0.1, iters=300):
    """Image i of the batched workload: sides U{lo..hi}, lambda U[1, 20], delta frac*max|f|."""
    seed = 1000 + i
    rng = np.random.default_rng(seed)
    H = int(rng.integers(lo, hi + 1))
    W = int(rng.integers(lo, hi + 1))
    lam = float(rng.uniform(1.0, 20.0))
    z, mask = disc_rect_image(H, W, seed)
    prob = _finish(z, mask, 0.8, 0.2, lam=lam, iters=iters, meta=dict(name="disc_rect", seed=seed))
    prob.delta = band_delta(prob.f, frac)
    return prob


def config4(n=512, lo=64, hi=1024, frac=0.1, iters=300) -> List[Problem]:
    return [config4_image(i, lo, hi, frac, iters) for i in range(n)]


def config5(size=2048, frac=0.1, iters=300, seed=11):
    """Differentiation workload: disc + rectangle at 2048^2, target = noise-free mask."""
    z, mask = disc_rect_image(size, size, seed)
    prob = _finish(z, mask, 0.8, 0.2, lam=5.0, iters=iters, meta=dict(name="disc_rect", seed=seed))
    prob.delta = band_delta(prob.f, frac)
    return prob


TAU3 = 1.0 / 12.0   # Chambolle's step bound with three gradient components


def ellipsoids_volume(D, H, W, n, seed, sigma=0.05):
    """n random ellipsoids (intensity U[0.6, 0.9]) on a U[0.1, 0.3] background,
    Gaussian noise sigma; returns (z, mask) in FP64."""
    rng = np.random.default_rng(seed)
    z = np.full((D, H, W), rng.uniform(0.1, 0.3))
    mask = np.zeros((D, H, W), bool)
    zz, yy, xx = np.mgrid[0:D, 0:H, 0:W].astype(np.float64)
    for _ in range(n):
        c = rng.uniform(0.2, 0.8, 3) * np.array([D, H, W])
        a = rng.uniform(0.08, 0.2, 3) * np.array([D, H, W])
        inside = (((zz - c[0]) / a[0]) ** 2 + ((yy - c[1]) / a[1]) ** 2 +
                  ((xx - c[2]) / a[2]) ** 2) <= 1.0
        z[inside] = rng.uniform(0.6, 0.9)
        mask |= inside
    z = z + rng.normal(0.0, sigma, (D, H, W))
    return z, mask


def config_volume(size=256, n=8, lam=5.0, frac=float("inf"), iters=100, seed=21):
    """Volume workload: ellipsoids in a size^3 volume with the eq. CV term
    (c1, c2 the region means)."""
    z, mask = ellipsoids_volume(size, size, size, n, seed)
    c1, c2 = _region_means(z, mask)
    prob = _finish(z, mask, c1, c2, lam=lam, iters=iters, tau=TAU3,
                   meta=dict(name="ellipsoids", seed=seed, size=size))
    prob.delta = band_delta(prob.f, frac)
    return prob


def smooth_field(H, W, seed, scale=1.0, noise=0.1, modes=4):
    """Random smooth field plus noise: f with bands of small |f| along curves.

    Used for generic parity cases (random shapes, ragged edges)."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    f = np.zeros((H, W))
    for _ in range(modes):
        ky, kx = rng.uniform(0.5, 3.0, 2) * 2 * np.pi / np.array([max(H, 2), max(W, 2)])
        ph = rng.uniform(0, 2 * np.pi)
        f += rng.uniform(0.3, 1.0) * np.sin(ky * y + kx * x + ph)
    f = scale * f / max(1e-12, np.abs(f).max()) + rng.normal(0.0, noise, (H, W))
    return f.astype(np.float32)
