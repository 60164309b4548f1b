"""Benchmark of the restricted-domain dual solver on one MI355X.

Workload (one step): the restricted-domain sweep on 1024x1024 synthetic
ellipse images -- lambda in {1, 5, 20} (one image per lambda), delta in
{inf, 0.5, 0.2, 0.05} * max|f|, 500 iterations each, FP32 -- i.e. 12 solves
through the C ABI with inputs resident in HBM.  The metric is active
pixel-updates per second over the whole step (sum over solves of |RD| times
iterations, divided by the step time).

Also reported on the same line:
  roofline      the dominant iteration-kernel instantiation (most kernel time in
                the step; a resident solve counts as one launch of its own
                kernel): algorithmic bytes (28 per active pixel-iteration)
                per launch over its average launch duration, from HIP events
                around every launch on its stream, in a separate pass over the
                same step; peak = 8 TB/s HBM;
  cpu_baseline  the FP64 oracle (single thread) on a bounded sample of the same
                sweep (every case, fewer iterations), in the same unit;
  sweep         per case: active fraction, GPU time, label mismatch against
                the delta = inf solve at the same lambda, speed-up over it;
  extras        the batched workload (512 images, sides 64..1024, 300
                iterations, one hipGraph) against 512 sequential solves, also
                at delta = inf; forward + adjoint ms of the 2048^2
                differentiation workload; the 4096^2 distance-selective solve.

`python bench.py --gpus N --steps K --warmup W`; only N = 1 is supported.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = 28
# forward + adjoint with checkpoints: forward 28, segment recompute 28, segment
# tape 12, reverse step 40 (stored state, adjoint state, accumulator, c) per
# active pixel-iteration
ADJ_BYTES_PER_UPDATE = 108
# FP32 operations of one active pixel-update (FMA counted as 2; sqrt,
# reciprocal, min and max as 1 each): divergence 3, u-step 2, v-step 3, w 2,
# gradient 2, |g| 4, 1 / (1 + tau |g|) 3, the two p components 6
FLOPS_PER_UPDATE = 25
# FP32 vector peak without packed instructions (the library is built without
# them): 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
FP32_PEAK_PACKED_TFLOPS = 157.3
# VALU issue of the chip: each SIMD takes 4 cycles for a full-rate wave64
# instruction and 16 for a quarter-rate one (square root, reciprocal)
N_SIMDS = 256 * 4
N_XCDS = 8
CLOCK_HZ = 2.4e9
DEFAULT_TUNE_CACHE = os.path.join(ROOT, "paper_1807_11534_amd", "tuning", "mi355x.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--cpu-iters", type=int, default=100,
                    help="iterations per case for the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--tune", default="cache", choices=["cache", "auto", "fixed"],
                    help="cache: the library's choice from the tuning cache file (--tune-cache); "
                         "auto: autotune each case; fixed: 64x64 tiles, 4 iterations/launch")
    ap.add_argument("--tune-cache", default=DEFAULT_TUNE_CACHE,
                    help="tuning cache (rdseg.tune_cache_save text) read with --tune cache")
    ap.add_argument("--save-tune-cache", metavar="PATH",
                    help="write the tuning cache after the sweep's autotuning (--tune auto)")
    ap.add_argument("--extras", default="all",
                    help="comma-separated subset of the extra workloads: " + ", ".join(EXTRAS) +
                    " (batched_512: the batched workload at the specified delta only)")
    ap.add_argument("--extras-only", action="store_true",
                    help="run only the selected extra workloads and print their JSON")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-sized buffer with torch (counter calibration)")
    ap.add_argument("--roofline-kernel", metavar="NAME",
                    help="report the roofline of this iteration-kernel instantiation (as named "
                         "in roofline.kernel) instead of the one with the most time in the step "
                         "(counter runs, where the profiler's per-dispatch cost reorders them)")
    ap.add_argument("--maps-at-exit", metavar="PATH",
                    help="write /proc/self/maps to PATH at interpreter exit (attributes the "
                         "addresses of a crash in the process's exit handlers to the mapped "
                         "files)")
    return ap.parse_args()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed(torch, fn, reps=1):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def sweep_cases(torch, rdseg, synth, args, dev):
    probs = [synth.config2(i, size=args.size, iters=args.iters) for i in range(len(synth.C2_LAMBDAS))]
    cases = []
    for li, prob in enumerate(probs):
        f_dev = torch.from_numpy(prob.f).to(dev)
        for fr in synth.C2_FRACS:
            delta = synth.band_delta(prob.f, fr)
            q = float((np.abs(prob.f.astype(np.float64)) < delta).mean())
            cases.append(dict(li=li, lam=prob.lam, frac=fr, delta=delta, q=q, f=f_dev,
                              f_host=prob.f))
    for c in cases:
        f = c["f"]
        H, W = f.shape
        c["out"] = (torch.empty((H, W), device=dev), torch.empty((H, W), device=dev),
                    torch.empty((2, H, W), device=dev))
        c["ws"] = rdseg.workspace(rdseg.shape_of(f))
        if args.tune == "auto":
            tuned = rdseg.autotune(f, c["lam"], synth.THETA, synth.TAU, c["delta"], args.iters)
            (tile, ipl), comps, res = tuned, tuned.components, tuned.resident
        elif args.tune == "cache":
            # what a solve that leaves the choice to the library runs, given
            # the cache: every run with the same file times the same launches
            tuned = rdseg.tune_lookup(f.shape, c["q"])
            (tile, ipl), comps, res = tuned, tuned.components, tuned.resident
        else:
            tile, ipl, comps, res = (64, 64), 4, 0, 0
        c["tile"], c["ipl"], c["comps"], c["res"] = tile, ipl, comps, res
    if args.tune == "auto" and args.save_tune_cache:
        rdseg.tune_cache_save(args.save_tune_cache)
    return probs, cases


def protocol(torch, rdseg, synth, dev):
    """The evaluation protocol of Sec. 4 on synthetic stand-ins of the paper's
    three 128^2 examples (two eq. CV terms, one eq. DS term): ground truth from
    the unrestricted solve stopped at a change of 1e-10 (or 20000 iterations),
    then for q = 0, 0.1, ..., 1 the restricted solve with q-hat from q, stopped
    at 1e-2 (checked every iteration); E1, E2 against the ground truth,
    iterations and wall time (q-hat selection included)."""
    cases = [("disc_rect_cv", synth.config1()),
             ("ellipses_cv", synth.config2(1, 128, 500)),
             ("blobs_ds", synth.config3(size=128))]
    out = {}
    for name, pr in cases:
        log(f"extras: protocol {name}")
        f = torch.from_numpy(pr.f).to(dev)
        ws = rdseg.workspace(rdseg.shape_of(f))
        ugt, _, _, done_gt, d_gt = rdseg.solve_until(f, pr.lam, synth.THETA, synth.TAU, math.inf,
                                                     20000, 1e-10, 1, tile=(16, 16),
                                                     iters_per_launch=1, ws=ws)
        ugt = ugt.clone()
        n_gt = int(done_gt.item())
        rows = []
        for q in [round(0.1 * k, 1) for k in range(11)]:
            def run():
                delta = rdseg.band_threshold(f, q)
                dq = float(delta.item())
                return dq, rdseg.solve_until(f, pr.lam, synth.THETA, synth.TAU, dq, 20000, 1e-2,
                                             1, tile=(16, 16), iters_per_launch=1, ws=ws)
            run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dq, (u, v, p, done, _) = run()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            e1, e2 = rdseg.e1_e2(u, ugt)
            rows.append(dict(q=q, qhat=dq, iters=int(done.item()), ms=round(ms, 3),
                             E1=round(e1, 5), E2=float(f"{e2:.4g}")))
        out[name] = dict(size=list(pr.f.shape), lam=pr.lam, gt_iters=n_gt,
                         gt_last_change=float(d_gt[n_gt - 1].item()) if n_gt else None,
                         rows=rows)
    return out


EXTRAS = ("batched", "adjoint", "protocol", "primal_dual", "volume", "ds_4096")


def extras(torch, rdseg, synth, dev, which=EXTRAS):
    out = {}
    if "batched" in which or "batched_512" in which:
        # ---- batched workload: 512 images, sides 64..1024, 300 iterations
        # ("batched_512": the specified delta only)
        log("extras: generating the batched workload")
        probs = synth.config4(512, frac=0.1)
        runs = [(0.1, "batched_512"), (math.inf, "batched_512_delta_inf")]
        for frac, name in (runs if "batched" in which else runs[:1]):
            log(f"extras: {name}")
            fs = [torch.from_numpy(p.f).to(dev) for p in probs]
            lams = [p.lam for p in probs]
            deltas = [p.delta if math.isfinite(frac) else math.inf for p in probs]
            n_px = sum(p.f.size for p in probs)
            q = sum(float((np.abs(p.f.astype(np.float64)) < d).sum())
                    for p, d in zip(probs, deltas)) / n_px
            # the library's choice for the batch (configuration and form of
            # the iterations from the committed tuning cache's entry for the
            # batch's class, written by rdseg_autotune_batched runs on this
            # workload), captured as one graph
            bs = rdseg.BatchedSolver(fs, lams, deltas, synth.THETA, synth.TAU, 300, tile=None,
                                     iters_per_launch=0, graph=True)
            tuned = bs.lookup(q)
            (tile, ipl), form = tuned, tuned.form
            reps = 2 if not math.isfinite(frac) else 10
            bs.run()
            bs.run()
            t_graph = timed(torch, bs.run, reps)
            outs = [tuple(t.clone() for t in o) for o in bs.out]
            seq_out = [tuple(torch.empty_like(t) for t in o) for o in bs.out]
            wss = [rdseg.workspace(rdseg.shape_of(f)) for f in fs]

            def sequential():
                for i, f in enumerate(fs):
                    rdseg.solve(f, lams[i], synth.THETA, synth.TAU, deltas[i], 300, tile=tile,
                                iters_per_launch=ipl, out=seq_out[i], ws=wss[i])

            sequential()
            t_seq = timed(torch, sequential, 3)
            same = all(torch.equal(a[0], b[0]) for a, b in zip(outs, seq_out))
            upd = q * n_px * 300
            forms = {1: "persistent", 2: "launches"}
            out[name] = dict(images=512, pixels=n_px, active_fraction=q, iters=300,
                             tile=list(tile), iters_per_launch=ipl, form=forms[form],
                             configuration="tuning cache" if tuned.cached else "untuned default",
                             graph_ms=t_graph,
                             sequential_ms=t_seq, speedup=t_seq / t_graph,
                             updates_per_s=upd / (t_graph * 1e-3),
                             bitwise_equal_to_sequential=bool(same))
            bs.close()
            del fs, outs, seq_out, wss, bs
            torch.cuda.empty_cache()
    if "adjoint" in which:
        # ---- differentiation workload: 2048^2, 300 iterations, checkpoints every 30
        prob = synth.config5()
        f = torch.from_numpy(prob.f).to(dev)
        tgt = torch.from_numpy(prob.mask.astype(np.float32)).to(dev)
        for frac, name in [(0.1, "fwd_adjoint_2048"), (0.5, "fwd_adjoint_2048_delta_0.5")]:
            log(f"extras: {name}")
            delta = synth.band_delta(prob.f, frac)
            q = float((np.abs(prob.f.astype(np.float64)) < delta).mean())

            def fwd_bwd():
                u, v, p, tape = rdseg.solve(f, prob.lam, synth.THETA, synth.TAU, delta, 300,
                                            ckpt_every=30)
                rdseg.backward(f, prob.lam, synth.THETA, synth.TAU, delta, 300, 30, tape,
                               2 * (u - tgt))

            def fwd_only():   # the untaped forward in the library's own configuration
                rdseg.solve(f, prob.lam, synth.THETA, synth.TAU, delta, 300)

            fwd_bwd()
            t_fb = timed(torch, fwd_bwd, 3)
            fwd_only()
            t_f = timed(torch, fwd_only, 3)
            alg = ADJ_BYTES_PER_UPDATE * q * 2048 * 2048 * 300
            # what the timed computation is checked against (tests/)
            checked = ("grad_f within 1e-3 of the FP64 reverse on sampled component crops at "
                       "these 300 iterations; every reverse form bitwise equal"
                       if frac == 0.1 else
                       "the exact reverse of the FP32 forward (every reverse form and the "
                       "component path bitwise equal); FP64-reverse parity 1e-3 on a 64x64 crop "
                       "of the 512^2 image of this workload at 200 iterations only: at 300 the "
                       "reverse sweep is ill-conditioned where the dual field has converged "
                       "(rounding-level gradients set its direction)")
            out[name] = dict(size=2048, iters=300, ckpt_every=30, active_fraction=q,
                             checked=checked, fwd_adjoint_ms=t_fb, forward_ms=t_f,
                             alg_bytes_per_update=ADJ_BYTES_PER_UPDATE,
                             # unblocked-equivalent: the component path keeps its
                             # chains on chip, so this can exceed the HBM peak
                             alg_gbs=alg / (t_fb * 1e-3) / 1e9)
        del f, tgt
    if "protocol" in which:
        out["paper_protocol_128"] = protocol(torch, rdseg, synth, dev)
    if "primal_dual" in which:
        # ---- restricted primal-dual solve of eq. CR on the 1024^2 sweep image
        prob = synth.config2(1, 1024, 500)
        f = torch.from_numpy(prob.f).to(dev)
        for frac, name in [(math.inf, "primal_dual_1024_delta_inf"),
                           (0.5, "primal_dual_1024_delta_0.5")]:
            log(f"extras: {name}")
            delta = synth.band_delta(prob.f, frac)
            q = float((np.abs(prob.f.astype(np.float64)) < delta).mean())
            outp = (torch.empty_like(f), torch.empty((2,) + tuple(f.shape), dtype=torch.float32,
                                                     device=dev))
            wsp = torch.empty(rdseg._lib.load().rdseg_pd_workspace_size(
                rdseg.ctypes.byref(rdseg.shape_of(f))), dtype=torch.uint8, device=dev)
            run = lambda: rdseg.solve_pd(f, prob.lam, delta, 500, out=outp, ws=wsp)
            run()
            t = timed(torch, run, 3)
            upd = q * prob.f.size * 500
            out[name] = dict(size=1024, iters=500, active_fraction=q, ms=t,
                             updates_per_s=upd / (t * 1e-3),
                             alg_gbs=36.0 * upd / (t * 1e-3) / 1e9)
            del outp, wsp
        del f
    if "volume" in which:
        # ---- 256^3 volume (7-point stencil), 100 iterations
        prob = synth.config_volume(256)
        f = torch.from_numpy(prob.f).to(dev)
        for frac, name in [(math.inf, "volume_256_delta_inf"), (0.2, "volume_256_delta_0.2")]:
            log(f"extras: {name}")
            delta = synth.band_delta(prob.f, frac)
            q = float((np.abs(prob.f.astype(np.float64)) < delta).mean())
            out3 = (torch.empty_like(f), torch.empty_like(f),
                    torch.empty((3,) + tuple(f.shape), dtype=torch.float32, device=dev))
            ws = torch.empty(rdseg._lib.load().rdseg_workspace_size3(
                rdseg.ctypes.byref(rdseg.shape3_of(f))), dtype=torch.uint8, device=dev)
            run = lambda: rdseg.solve3d(f, prob.lam, synth.THETA, synth.TAU3, delta, 100, out=out3,
                                        ws=ws)
            run()
            t = timed(torch, run, 3)
            upd = q * prob.f.size * 100
            out[name] = dict(size=[256, 256, 256], iters=100, active_fraction=q, ms=t,
                             updates_per_s=upd / (t * 1e-3),
                             alg_gbs=36.0 * upd / (t * 1e-3) / 1e9)
            del ws, out3
        del f
        torch.cuda.empty_cache()
    if "ds_4096" in which:
        # ---- 4096^2 distance-selective solve, delta 0.1 max|f|, 1000 iterations
        log("extras: ds_4096")
        prob = synth.config3()
        f = torch.from_numpy(prob.f).to(dev)
        q = float((np.abs(prob.f.astype(np.float64)) < prob.delta).mean())
        # the persistent kernel at 8 iterations per launch, tile autotuned;
        # the unrestricted autotuner's pick is timed beside it
        res = {}
        for key, fixed in (("ipl8", 8), ("free", 0)):
            tuned = rdseg.autotune(f, prob.lam, synth.THETA, synth.TAU, prob.delta, 200,
                                   iters_per_launch=fixed)
            (tile, ipl), comps, resv = tuned, tuned.components, tuned.resident
            run = lambda: rdseg.solve(f, prob.lam, synth.THETA, synth.TAU, prob.delta, 1000,
                                      tile=tile, iters_per_launch=ipl, components=comps,
                                      resident=resv)
            run()
            t = timed(torch, run, 2)
            res[key] = dict(ms=t, tile=list(tile), iters_per_launch=ipl,
                            small_components={1: "on", 2: "off"}[comps],
                            barrier={1: "on-chip", 2: "launches"}[resv],
                            updates_per_s=q * prob.f.size * 1000 / (t * 1e-3))
        out["ds_4096"] = dict(size=4096, iters=1000, active_fraction=q, **res["ipl8"],
                              autotuned_free=res["free"])
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(pass --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.maps_at_exit:
        import atexit

        def dump_maps(path=args.maps_at_exit):
            with open("/proc/self/maps") as src, open(path, "w") as dst:
                dst.write(src.read())
        atexit.register(dump_maps)   # registered first: runs after the binding's release
    import torch

    import synth
    from paper_1807_11534_amd import rdseg

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    which = EXTRAS if args.extras == "all" else tuple(x.strip() for x in args.extras.split(","))
    unknown = [x for x in which if x not in EXTRAS + ("batched_512",)]
    if unknown:
        print(f"unknown extra workloads: {unknown}; choose from {EXTRAS}", file=sys.stderr)
        sys.exit(2)
    if args.tune == "cache":
        if not os.path.exists(args.tune_cache):
            print(f"tuning cache {args.tune_cache} not found (make one with --tune auto "
                  f"--save-tune-cache PATH)", file=sys.stderr)
            sys.exit(2)
        rdseg.tune_cache_clear()
        rdseg.tune_cache_load(args.tune_cache)
    if args.extras_only:
        print(json.dumps(dict(extras=extras(torch, rdseg, synth, dev, which))), flush=True)
        return
    log("sweep: generating and tuning")
    probs, cases = sweep_cases(torch, rdseg, synth, args, dev)

    def step():
        for c in cases:
            rdseg.solve(c["f"], c["lam"], synth.THETA, synth.TAU, c["delta"], args.iters,
                        tile=c["tile"], iters_per_launch=c["ipl"], out=c["out"], ws=c["ws"],
                        components=c["comps"], resident=c["res"])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    n_px = args.size * args.size
    updates_per_step = sum(c["q"] * n_px * args.iters for c in cases)
    value = updates_per_step / (ms_per_step * 1e-3)

    # per-case detail (one more timed pass, per solve)
    detail = []
    ref_labels = {}
    for c in cases:
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        u, v, p = rdseg.solve(c["f"], c["lam"], synth.THETA, synth.TAU, c["delta"], args.iters,
                              tile=c["tile"], iters_per_launch=c["ipl"], out=c["out"], ws=c["ws"],
                              components=c["comps"], resident=c["res"])
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        lab = (u > 0.5).cpu().numpy()
        if not math.isfinite(c["frac"]):
            ref_labels[c["li"]] = (lab, ms)
        ref_lab, ref_ms = ref_labels[c["li"]]
        detail.append(dict(lam=c["lam"], delta_frac=c["frac"] if math.isfinite(c["frac"]) else "inf",
                           q=round(c["q"], 6), ms=round(ms, 4),
                           updates_per_s=c["q"] * n_px * args.iters / (ms * 1e-3),
                           label_mismatch_vs_inf=float((lab != ref_lab).mean()),
                           speedup_vs_inf=round(ref_ms / ms, 3),
                           tile=list(c["tile"]), iters_per_launch=c["ipl"],
                           small_components={1: "on", 2: "off"}.get(c["comps"], "default"),
                           barrier={1: "on-chip", 2: "launches"}.get(c["res"], "default")))

    # roofline pass: HIP events around every iteration-kernel launch; the last
    # GPU work before the extras, so that its launches are the last dispatches of
    # their kernels in a profiler trace of a run without extras
    rdseg.timing_reset()
    rdseg.timing_enable(True)
    step()
    torch.cuda.synchronize()
    rdseg.timing_enable(False)
    cfgs = rdseg.configs()
    per_cfg = []
    for ci, (tw, th, it, nt) in enumerate(cfgs):
        # form 0: separate launches of the blocked kernel; 1: resident launches
        for form, name in ((0, "k_iterate"), (1, "k_resident")):
            ms, nl, by, upd = rdseg.timing_read_form(ci, form)
            if nl:
                per_cfg.append(dict(config=ci, kernel=f"{name}<{tw},{th},{it},{nt}>", ms=ms,
                                    launches=nl, alg_bytes=by, updates=upd))
    if args.roofline_kernel:
        named = [r for r in per_cfg if r["kernel"] == args.roofline_kernel]
        if not named:
            print(f"--roofline-kernel {args.roofline_kernel}: not launched in the step "
                  f"(launched: {[r['kernel'] for r in per_cfg]})", file=sys.stderr)
            sys.exit(2)
        dom = named[0]
    else:
        dom = max(per_cfg, key=lambda r: r["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    bytes_per_launch = dom["alg_bytes"] / dom["launches"]
    updates_per_launch = dom["updates"] / dom["launches"]
    alg_gbs = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    achieved = FLOPS_PER_UPDATE * updates_per_launch / (avg_ms * 1e-3) / 1e12
    all_ms, all_n, all_b, _ = rdseg.timing_read(-1)
    rdseg.timing_reset()

    ext = None
    if not args.no_extras:
        ext = extras(torch, rdseg, synth, dev, which)

    cpu = None
    if not args.no_cpu:
        import oracle
        log("cpu baseline: oracle sample")
        t0 = time.perf_counter()
        upd = 0.0
        for c in cases:
            oracle.solve(c["f_host"], c["lam"], synth.THETA, synth.TAU, c["delta"], args.cpu_iters)
            upd += c["q"] * n_px * args.cpu_iters
        dt = time.perf_counter() - t0
        cpu = dict(value=upd / dt, unit="active pixel-updates/s", cores=1, kind="oracle",
                   sample=f"all 12 sweep cases at {args.size}^2, {args.cpu_iters} iterations each "
                          f"(FP64, single thread), {dt:.1f} s; the oracle sweeps the whole grid "
                          f"every iteration (frozen pixels included), so the sparse bands are "
                          f"charged full-grid work",
                   cpu_model=cpu_model(), host_cpus=os.cpu_count())

    # HBM bytes and instruction counts per launch of the dominant kernel from
    # the counter passes recorded under profiles/ (FETCH_SIZE + WRITE_SIZE,
    # copy-calibrated; SQ instruction counters), only when they were taken
    # from the current kernel sources
    from paper_1807_11534_amd.profiling import recorded_counters, recorded_traffic
    prof_dir = os.path.join(ROOT, "profiles")
    rec = recorded_traffic(dom["kernel"], prof_dir)
    traffic = rec[0] if rec else None
    sq = recorded_counters(dom["kernel"], prof_dir)
    valu = None
    if sq:
        cnt, src = sq
        insts = cnt.get("SQ_INSTS_VALU")
        trans = cnt.get("SQ_INSTS_VALU_TRANS_F32", 0.0)
        if insts:
            # SIMD cycles of VALU issue: 4 per full-rate wave64 instruction,
            # 16 per quarter-rate one, over all SIMDs for this run's launch
            # duration at the nominal clock
            cycles = 4.0 * (insts - trans) + 16.0 * trans
            valu = dict(insts_per_launch=insts, trans_insts_per_launch=trans,
                        issue_frac=cycles / (N_SIMDS * CLOCK_HZ * avg_ms * 1e-3),
                        lane_insts_per_update=insts * 64.0 / updates_per_launch,
                        counters=cnt, source=src)
            act, gui = cnt.get("SQ_ACTIVE_INST_VALU"), cnt.get("GRBM_GUI_ACTIVE")
            if act and gui:
                # within the counter run: VALU-busy SIMD cycles (the counter is
                # in quad-cycles) over all SIMDs for the dispatch's GPU cycles
                # (GRBM_GUI_ACTIVE sums the 8 XCDs)
                valu["busy_frac"] = 4.0 * act / (N_SIMDS * gui / N_XCDS)

    line = dict(
        metric="active pixel-updates/s (restricted-domain sweep)",
        value=value,
        unit="active pixel-updates/s",
        n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=ms_per_step,
        higher_is_better=True,
        scaling="weak",
        vs_baseline=None,
        dtype="f32",
        data="synthetic",
        config=dict(workload=f"restricted-domain sweep, {args.size}x{args.size} ellipse images, "
                             f"lambda {{1,5,20}} x delta {{inf,0.5,0.2,0.05}}*max|f|, "
                             f"{args.iters} iterations",
                    images=len(probs), solves_per_step=len(cases),
                    pixel_updates_per_step=updates_per_step),
        roofline=dict(bound="alu", achieved=achieved, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                      frac=achieved / FP32_PEAK_TFLOPS, traffic=traffic,
                      traffic_source=rec[1] if rec else None,
                      kernel=dom["kernel"], launches=dom["launches"], avg_launch_ms=avg_ms,
                      flops_per_update=FLOPS_PER_UPDATE, updates_per_launch=updates_per_launch,
                      frac_of_packed_peak=achieved / FP32_PEAK_PACKED_TFLOPS,
                      valu=valu,
                      hbm=dict(alg_bytes_per_update=BYTES_PER_UPDATE,
                               alg_bytes_per_launch=bytes_per_launch, alg_gbs=alg_gbs,
                               alg_frac=alg_gbs / HBM_PEAK_GBS,
                               traffic_gbs=(traffic / (avg_ms * 1e-3) / 1e9) if traffic else None,
                               traffic_frac=(traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
                               if traffic else None, peak=HBM_PEAK_GBS),
                      all_iterate_launches=dict(launches=all_n, ms=all_ms,
                                                gbs=all_b / (all_ms * 1e-3) / 1e9 if all_ms else 0.0),
                      per_config=per_cfg),
        cpu_baseline=cpu,
        sweep=detail,
        extras=ext,
    )
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
