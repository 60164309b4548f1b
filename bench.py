"""Benchmark of the restricted-domain dual solver on one MI355X.

Workload (one step): the restricted-domain sweep on 1024x1024 synthetic
ellipse images -- lambda in {1, 5, 20} (one image per lambda), delta in
{inf, 0.5, 0.2, 0.05} * max|f|, 500 iterations each, FP32 -- i.e. 12 solves
through the C ABI with inputs resident in HBM.  The metric is active
pixel-updates per second over the whole step (sum over solves of |RD| times
iterations, divided by the step time).

Also reported on the same line:
  roofline      achieved algorithmic HBM bytes per second of the iteration
                kernel (28 bytes per active pixel-iteration), measured with HIP
                events around every launch of that kernel in a separate pass
                over the same step, against the 8 TB/s HBM peak;
  cpu_baseline  the FP64 oracle (single thread) on a bounded sample of the same
                sweep (every case, fewer iterations), in the same unit;
  sweep         per case: active fraction, GPU time, label mismatch against
                the delta = inf solve at the same lambda, speed-up over it.

`python bench.py --gpus N --steps K --warmup W`; only N = 1 is supported (the
build runs on one GPU).
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--cpu-iters", type=int, default=30,
                    help="iterations per case for the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune", default="auto", choices=["auto", "fixed"],
                    help="auto: autotune each case; fixed: 64x64 tiles, 4 iterations/launch")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(pass --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_1807_11534_amd import rdseg

    dev = torch.device("cuda:0")
    lams = synth.C2_LAMBDAS
    fracs = synth.C2_FRACS
    probs = [synth.config2(i, size=args.size, iters=args.iters) for i in range(len(lams))]
    cases = []
    for li, prob in enumerate(probs):
        f_dev = torch.from_numpy(prob.f).to(dev)
        for fr in fracs:
            delta = synth.band_delta(prob.f, fr)
            q = float((np.abs(prob.f.astype(np.float64)) < delta).mean())
            cases.append(dict(li=li, lam=prob.lam, frac=fr, delta=delta, q=q, f=f_dev,
                              f_host=prob.f))
    # preallocate outputs and workspaces (inputs and state resident in HBM)
    for c in cases:
        f = c["f"]
        H, W = f.shape
        c["out"] = (torch.empty((H, W), device=dev), torch.empty((H, W), device=dev),
                    torch.empty((2, H, W), device=dev))
        c["ws"] = rdseg.workspace(rdseg.shape_of(f))
        if args.tune == "auto":
            tile, ipl = rdseg.autotune(f, c["lam"], synth.THETA, synth.TAU, c["delta"], 16)
        else:
            tile, ipl = (64, 64), 4
        c["tile"], c["ipl"] = tile, ipl

    def step():
        for c in cases:
            rdseg.solve(c["f"], c["lam"], synth.THETA, synth.TAU, c["delta"], args.iters,
                        tile=c["tile"], iters_per_launch=c["ipl"], out=c["out"], ws=c["ws"])

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

    # roofline pass: HIP events around every iteration-kernel launch
    rdseg.timing_enable(True)
    step()
    torch.cuda.synchronize()
    k_ms, k_launch, k_bytes, k_upd = rdseg.timing_read()
    rdseg.timing_enable(False)
    achieved = k_bytes / (k_ms * 1e-3) / 1e9 if k_ms > 0 else 0.0

    # per-case detail (one more timed pass, per solve)
    detail = []
    ref_labels = {}
    for c in cases:
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        u, v, p = rdseg.solve(c["f"], c["lam"], synth.THETA, synth.TAU, c["delta"], args.iters,
                              tile=c["tile"], iters_per_launch=c["ipl"], out=c["out"], ws=c["ws"])
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
                           tile=list(c["tile"]), iters_per_launch=c["ipl"]))

    cpu = None
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        upd = 0.0
        for c in cases:
            oracle.solve(c["f_host"], c["lam"], synth.THETA, synth.TAU, c["delta"], args.cpu_iters)
            upd += c["q"] * n_px * args.cpu_iters
        dt = time.perf_counter() - t0
        cpu = dict(value=upd / dt, unit="active pixel-updates/s", cores=1, kind="oracle",
                   sample=f"all 12 sweep cases at {args.size}^2, {args.cpu_iters} iterations each "
                          f"(FP64, single thread), {dt:.1f} s")

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
        roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS, traffic=None,
                      kernel="k_iterate", launches=k_launch, kernel_ms=k_ms,
                      alg_bytes_per_update=BYTES_PER_UPDATE),
        cpu_baseline=cpu,
        sweep=detail,
    )
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
