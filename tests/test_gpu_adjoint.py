"""Adjoint kernels (through the C ABI): against the FP64 reverse-mode oracle on
64x64 crops, against central finite differences of the GPU forward, the
fitting-term kernels against the oracle, and the autograd composition.

Bar: relative error <= 1e-3, with the error of a gradient field measured as
max|g_gpu - g_ref| / max|g_ref| and of a scalar as |g_gpu - g_ref| / |g_ref|.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
REL = 1e-3


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def rd(gpu):
    from paper_1807_11534_amd import rdseg
    return rdseg


def boundary_crop(prob, size=64):
    """Crop centred on the disc's rightmost boundary point (scaled geometry)."""
    H, W = prob.f.shape
    cy = int(64 * H / 128)
    cx = int((40 + 30) * W / 128)
    y0 = min(max(cy - size // 2, 0), H - size)
    x0 = min(max(cx - size // 2, 0), W - size)
    return (slice(y0, y0 + size), slice(x0, x0 + size))


@pytest.mark.parametrize("frac,K", [(math.inf, 300), (0.1, 300), (0.5, 200)])
@pytest.mark.parametrize("with_v", [False, True])
def test_adjoint_vs_oracle_crop(rd, frac, K, with_v):
    """64x64 crop across the disc boundary.  delta = 0.5 max|f| runs 200
    iterations: at 300 its gradient is ill-conditioned in any FP32 arithmetic
    (the conditioning tests pin both facts)."""
    prob = synth.config5(size=512)
    sl = boundary_crop(prob)
    f = np.ascontiguousarray(prob.f[sl])
    target = prob.mask[sl].astype(np.float64)
    delta = synth.band_delta(f, frac)
    ce, lam = 30, prob.lam
    print(f"adjoint crop frac={frac} with_v={with_v}", flush=True)
    fd = dev(f)
    u, v, p, tape = rd.solve(fd, lam, 0.1, 0.125, delta, K, tile=(32, 32), iters_per_launch=2,
                             ckpt_every=ce)
    uo, vo, _ = oracle.solve(f, lam, 0.1, 0.125, delta, K)
    assert np.abs(host(u) - uo).max() <= 1e-4
    ub = 2 * (host(u).astype(np.float64) - target)
    rng = np.random.default_rng(9)
    vb = rng.normal(size=f.shape) if with_v else None
    gu = dev(ub.astype(np.float32))
    gv = dev(vb.astype(np.float32)) if with_v else None
    gf, gl = rd.backward(fd, lam, 0.1, 0.125, delta, K, ce, tape, gu, gv)
    fbo, lbo = oracle.reverse(f, lam, 0.1, 0.125, delta, K, host(gu).astype(np.float64),
                              None if vb is None else host(gv).astype(np.float64))
    g = host(gf).astype(np.float64)
    scale = max(np.abs(fbo).max(), 1e-12)
    assert np.abs(g - fbo).max() <= REL * scale, (np.abs(g - fbo).max(), scale)
    lg = float(host(gl))
    assert abs(lg - lbo) <= REL * max(abs(lbo), 1e-9), (lg, lbo)
    A = np.abs(f.astype(np.float64)) < delta
    assert (g[~A] == 0).all()


def test_adjoint_deterministic_and_ipl_invariant(rd):
    prob = synth.config5(size=256)
    f = prob.f
    delta = synth.band_delta(f, 0.5)
    fd = dev(f)
    outs = []
    for (tile, ipl) in [((32, 32), 2), ((64, 64), 4), ((16, 16), 1)]:
        u, v, p, tape = rd.solve(fd, 5.0, 0.1, 0.125, delta, 95, tile=tile, iters_per_launch=ipl,
                                 ckpt_every=30)
        gu = 2 * (u - dev(prob.mask.astype(np.float32)))
        gf, gl = rd.backward(fd, 5.0, 0.1, 0.125, delta, 95, 30, tape, gu)
        outs.append((host(gf), float(host(gl))))
    for o in outs[1:]:
        np.testing.assert_array_equal(o[0], outs[0][0])
        assert o[1] == outs[0][1]


def test_adjoint_vs_finite_differences(rd):
    """GPU adjoint against central differences of the FP64 forward on the 16
    pixels of the restricted domain and its one-ring with the largest gradient
    (step 2^-20, exact in FP32) and on lambda (step 1e-6).  The unrolled map is
    only piecewise smooth (clamp, and |g| at g = 0), so the step must stay below
    the distance to the nearest kink: 1e-3 is not, at this crop.  The domain and
    u0 are held fixed by keeping |f| and ||f| - delta| above 2h at those pixels.
    Differences of the FP32 forward itself are not used: a pixel step changes
    the loss by ~2h|g|, below the FP32 rounding noise of the loss."""
    prob = synth.config5(size=512)
    sl = boundary_crop(prob, 64)
    f = np.ascontiguousarray(prob.f[sl])
    target = prob.mask[sl].astype(np.float64)
    delta = synth.band_delta(f, 0.5)
    K, ce, lam, h = 200, 30, 5.0, 2.0 ** -20
    fd = dev(f)
    u, v, p, tape = rd.solve(fd, lam, 0.1, 0.125, delta, K, tile=(32, 32), iters_per_launch=2,
                             ckpt_every=ce)
    uo, _, _ = oracle.solve(f, lam, 0.1, 0.125, delta, K)
    ub = 2 * (uo - target)
    gf, gl = rd.backward(fd, lam, 0.1, 0.125, delta, K, ce, tape, dev(ub.astype(np.float32)))
    g = host(gf).astype(np.float64)
    ub32 = ub.astype(np.float32).astype(np.float64)

    def loss(ff, ll):
        uu, _, _ = oracle.solve(ff, ll, 0.1, 0.125, delta, K)
        return float((ub32 * uu).sum())   # linearised loss: its gradient is J^T ubar

    fbo, _ = oracle.reverse(f, lam, 0.1, 0.125, delta, K, ub32)
    A = np.abs(f.astype(np.float64)) < delta
    ring = A.copy()
    ring[1:, :] |= A[:-1, :]
    ring[:-1, :] |= A[1:, :]
    ring[:, 1:] |= A[:, :-1]
    ring[:, :-1] |= A[:, 1:]
    ok = ring & (np.abs(f) > 2 * h) & (np.abs(np.abs(f) - delta) > 2 * h)
    cand = np.argwhere(ok)
    order = np.argsort(-np.abs(fbo[ok]))
    pick = cand[order[:16]]
    gmax = np.abs(g).max()
    errs = []
    for (y, x) in pick:
        fp, fm = f.copy(), f.copy()
        fp[y, x] += np.float32(h)
        fm[y, x] -= np.float32(h)
        step = float(fp[y, x]) - float(fm[y, x])
        fdv = (loss(fp, lam) - loss(fm, lam)) / step
        errs.append((abs(g[y, x] - fdv) / max(abs(fdv), 1e-3 * gmax), int(y), int(x), g[y, x], fdv))
    hl = 1e-6
    fdl = (loss(f, lam + hl) - loss(f, lam - hl)) / (2 * hl)
    lg = float(host(gl))
    lerr = abs(lg - fdl) / max(abs(fdl), 1e-12)
    print("fd errors", sorted(errs, reverse=True)[:4], "lambda", lg, fdl, lerr, flush=True)
    assert max(e[0] for e in errs) <= REL, errs
    assert lerr <= REL, (lg, fdl)


def test_fit_term_kernels(rd):
    prob = synth.config3(size=256, iters=10)
    z, P = prob.z, prob.P
    f = rd.fit_forward(dev(z), prob.c1, prob.c2, prob.gamma, dev(P))
    fo = oracle.fit_term(z, prob.c1, prob.c2, prob.gamma, P)
    np.testing.assert_array_equal(host(f), fo.astype(np.float32))
    rng = np.random.default_rng(3)
    gfv = rng.normal(size=z.shape).astype(np.float32)
    a, b, c = rd.fit_backward(dev(z), prob.c1, prob.c2, dev(gfv), dev(P))
    ao, bo, co = oracle.fit_vjp(z, prob.c1, prob.c2, gfv.astype(np.float64), P)
    for x, y in [(a, ao), (b, bo), (c, co)]:
        assert abs(float(host(x)) - y) <= 1e-9 * max(1.0, abs(y))


def test_fused_fit_backward_matches_composition(rd):
    prob = synth.config5(size=256)
    z = dev(prob.z)
    f = rd.fit_forward(z, prob.c1, prob.c2, 0.0)
    delta = synth.band_delta(host(f), 0.5)
    u, v, p, tape = rd.solve(f, 5.0, 0.1, 0.125, delta, 60, tile=(32, 32), iters_per_launch=2,
                             ckpt_every=30)
    gu = 2 * (u - dev(prob.mask.astype(np.float32)))
    gf, gl, g1, g2, gg = rd.backward(f, 5.0, 0.1, 0.125, delta, 60, 30, tape, gu,
                                     fit=(z, None, prob.c1, prob.c2, 0.0))
    a, b, _ = rd.fit_backward(z, prob.c1, prob.c2, gf)
    for x, y in [(g1, a), (g2, b)]:
        xv, yv = float(host(x)), float(host(y))
        assert abs(xv - yv) <= 1e-5 * max(1e-9, abs(yv)), (xv, yv)


def test_autograd_end_to_end(rd):
    """FitTerm -> RDSolve -> sum (u - target)^2, against the oracle chain
    (fit_term -> reverse -> fit_vjp) on a 64x64 crop."""
    from paper_1807_11534_amd.autograd import FitTerm, RDSolve
    prob = synth.config5(size=512)
    sl = boundary_crop(prob)
    z = np.ascontiguousarray(prob.z[sl])
    target = prob.mask[sl].astype(np.float32)
    c1 = torch.tensor(prob.c1, dtype=torch.float64, requires_grad=True)
    c2 = torch.tensor(prob.c2, dtype=torch.float64, requires_grad=True)
    lam = torch.tensor(5.0, dtype=torch.float64, requires_grad=True)
    zt = dev(z)
    f = FitTerm.apply(zt, c1, c2, 0.0, None)
    fo = oracle.fit_term(z, prob.c1, prob.c2).astype(np.float32)
    np.testing.assert_array_equal(host(f), fo)
    delta = synth.band_delta(fo, 0.5)
    u = RDSolve.apply(f, lam, 0.1, 0.125, delta, 120, 30)
    loss = ((u - dev(target)) ** 2).sum()
    loss.backward()
    uo, _, _ = oracle.solve(fo, 5.0, 0.1, 0.125, delta, 120)
    fbo, lbo = oracle.reverse(fo, 5.0, 0.1, 0.125, delta, 120, 2 * (host(u).astype(np.float64) - target))
    a, b, _ = oracle.fit_vjp(z, prob.c1, prob.c2, fbo)
    assert abs(float(c1.grad) - a) <= REL * max(abs(a), 1e-9), (float(c1.grad), a)
    assert abs(float(c2.grad) - b) <= REL * max(abs(b), 1e-9), (float(c2.grad), b)
    assert abs(float(lam.grad) - lbo) <= REL * max(abs(lbo), 1e-9), (float(lam.grad), lbo)


def test_autograd_pitched_inputs(rd):
    """FitTerm -> RDSolve on planes with a row pitch above their width (views
    big[:, :W]) gives the gradients of the same chain on contiguous planes:
    incoming gradients are read with the pitch of f and z."""
    from paper_1807_11534_amd.autograd import FitTerm, RDSolve
    prob = synth.config5(size=512)
    sl = boundary_crop(prob)
    z = np.ascontiguousarray(prob.z[sl])
    H, W = z.shape
    target = dev(prob.mask[sl].astype(np.float32))
    grads = []
    for pitched in (False, True):
        if pitched:
            big = torch.zeros((H, W + 40), dtype=torch.float32, device="cuda")
            big[:, :W] = dev(z)
            zt = big[:, :W]
            assert zt.stride(0) == W + 40
        else:
            zt = dev(z)
        c1 = torch.tensor(prob.c1, dtype=torch.float64, requires_grad=True)
        c2 = torch.tensor(prob.c2, dtype=torch.float64, requires_grad=True)
        lam = torch.tensor(5.0, dtype=torch.float64, requires_grad=True)
        f = FitTerm.apply(zt, c1, c2, 0.0, None)
        delta = synth.band_delta(host(f), 0.5)
        u = RDSolve.apply(f, lam, 0.1, 0.125, delta, 90, 30)
        # an expanded weight makes the incoming gradient non-contiguous
        w = torch.ones((1, W), dtype=torch.float32, device="cuda").expand(H, W)
        loss = (w * (u - target) ** 2).sum()
        loss.backward()
        grads.append((float(c1.grad), float(c2.grad), float(lam.grad), host(u)))
    for a, b in zip(grads[0][:3], grads[1][:3]):
        assert a == b, (a, b)
    np.testing.assert_array_equal(grads[0][3], grads[1][3])


def test_backward_full_size_differentiation_workload(rd):
    """2048^2, 300 iterations, checkpoints every 30, delta 0.1 and 0.5 max|f|:
    deterministic, zero off the domain, finite."""
    prob = synth.config5()
    fd = dev(prob.f)
    tgt = dev(prob.mask.astype(np.float32))
    for frac in (0.1, 0.5):
        delta = synth.band_delta(prob.f, frac)
        print(f"full C5 frac={frac}", flush=True)
        res = []
        for _ in range(2):
            u, v, p, tape = rd.solve(fd, prob.lam, 0.1, 0.125, delta, 300, tile=(32, 32),
                                     iters_per_launch=2, ckpt_every=30)
            gf, gl = rd.backward(fd, prob.lam, 0.1, 0.125, delta, 300, 30, tape, 2 * (u - tgt))
            res.append((host(gf), float(host(gl))))
        np.testing.assert_array_equal(res[0][0], res[1][0])
        assert res[0][1] == res[1][1]
        A = np.abs(prob.f.astype(np.float64)) < delta
        assert (res[0][0][~A] == 0).all()
        assert np.isfinite(res[0][0]).all() and math.isfinite(res[0][1])


@pytest.mark.parametrize("case", [("config5_512", 0.1, 300, 30), ("config5_512", 0.5, 120, 30),
                                  ("ragged", 0.4, 90, 30), ("ragged", 0.4, 90, 7),
                                  ("ragged", 0.4, 130, 60), ("ragged", 0.4, 25, 30),
                                  ("config5_512", 0.5, 120, 100),
                                  ("config5_2048", 0.5, 60, 30), ("config5_2048", 0.5, 44, 30)])
def test_component_reverse_matches_tile_path(rd, case):
    """RD components of at most 256 pixels in both directions (those of 65-256
    pixels, the only ones above 64 at 2048^2 and delta = 0.5 max|f|, as groups
    of 128 / 256 lanes: the register form, or the per-pixel slots at
    ckpt_every 60 and 100): the component
    forward writes the same checkpoints (on RD, where the tape is defined) and
    the same u, v, p as the tile path, and their reverse sweep (all steps in
    one launch) gives the same bits as the tile path's per-step launches
    (with few waves, ckpt_every 7 and 30 keep each step's dual-update outputs
    in LDS, with a second wave running the next segment's forward when there
    are several segments; many waves or ckpt_every 60 keep the states; 100 the
    per-pixel slots; at 2048^2, ~35K waves, the register form: checkpoints
    every 8 states and each 8-step sub-segment's dual-update outputs in
    registers, ragged sub-segments included),
    with a fitting-term gradient and both adjoint inputs."""
    name, frac, K, ce = case
    if name == "config5_2048":
        prob = synth.config5(size=2048)
        f, z, target = prob.f, prob.z, prob.mask.astype(np.float32)
    elif name == "ragged":
        f = synth.smooth_field(173, 211, 45, noise=0.35)
        z = synth.smooth_field(173, 211, 46, noise=0.1)
        target = (f < 0).astype(np.float32)
    else:
        prob = synth.config5(size=512)
        f, z, target = prob.f, prob.z, prob.mask.astype(np.float32)
    delta = synth.band_delta(f, frac)
    A = np.abs(f.astype(np.float64)) < delta
    fd = dev(f)
    print(f"component forward / reverse {case}", flush=True)
    out = {}
    try:
        for on in (False, True):
            rd.set_components(on)
            u, v, p, tape = rd.solve(fd, 4.0, 0.1, 0.125, delta, K, tile=(32, 32),
                                     iters_per_launch=2, ckpt_every=ce)
            gu = 2 * (u - dev(target))
            gv = 0.5 * (v - dev(target))
            fit = (dev(z), None, 0.8, 0.2, 0.0)
            H, W = f.shape
            slots = host(tape).reshape(-1, 3, H, W)[:, :, A]
            out[on] = [host(u), host(v), host(p), slots] + [
                host(x) for x in rd.backward(fd, 4.0, 0.1, 0.125, delta, K, ce, tape, gu, gv,
                                             fit=fit)]
    finally:
        rd.set_components(True)
    for a, b in zip(out[True], out[False]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("case", [("config5_512", 0.5, 120, 30), ("config5_512", math.inf, 62, 30),
                                  ("ragged", 0.4, 90, 7), ("ragged", 0.4, 25, 30),
                                  ("ragged", math.inf, 33, 11)])
@pytest.mark.parametrize("components", [False, True])
def test_reverse_forms_bitwise(rd, case, components):
    """The reverse sweep's forms (steps per launch 1, 2 and 4 on 16x16 and
    32x32 macro tiles, ragged last launches of a segment included) give the
    same bits as one step per launch: every gradient output."""
    name, frac, K, ce = case
    if name == "ragged":
        f = synth.smooth_field(173, 211, 45, noise=0.35)
        z = synth.smooth_field(173, 211, 46, noise=0.1)
        target = (f < 0).astype(np.float32)
    else:
        prob = synth.config5(size=512)
        f, z, target = prob.f, prob.z, prob.mask.astype(np.float32)
    delta = synth.band_delta(f, frac) if math.isfinite(frac) else math.inf
    fd = dev(f)
    print(f"reverse forms {case} components={components}", flush=True)
    out = {}
    try:
        rd.set_components(components)
        u, v, p, tape = rd.solve(fd, 4.0, 0.1, 0.125, delta, K, tile=(32, 32),
                                 iters_per_launch=2, ckpt_every=ce)
        gu = 2 * (u - dev(target))
        gv = 0.5 * (v - dev(target))
        fit = (dev(z), None, 0.8, 0.2, 0.0)
        for form in ((32, 1), (16, 2), (16, 4), (32, 2), (32, 4)):
            rd.set_adjoint_form(*form)
            out[form] = [host(x) for x in rd.backward(fd, 4.0, 0.1, 0.125, delta, K, ce, tape,
                                                      gu, gv, fit=fit)]
    finally:
        rd.set_components(True)
        rd.set_adjoint_form(0, 0)
    ref = out[(32, 1)]
    assert np.abs(ref[0]).max() > 0
    for form, res in out.items():
        for a, b in zip(res, ref):
            np.testing.assert_array_equal(a, b, err_msg=str(form))
