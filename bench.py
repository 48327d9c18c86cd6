"""Benchmark: full Dykstra projection of one 1024x1024 FP32 residual image.

Workload (the paper's test images are not available; a seeded synthetic frame
of the same kind stands in): 2000 point emitters, Poisson(50) counts, Gaussian
PSF sigma 1.5 px, minus the blurred mean, unit variance; windows of side
1..16 at every position; bounds = chi-square(s^2) 0.9 quantiles; FP32 image
and increments, Kahan window sums, FP64 convergence check, tol 1e-5 on the
largest pixel change per sweep.

A step is one projection to tolerance of that image (time-to-tol), starting
from the image resident in HBM.  value = window projections per second
(windows x sweeps / time).  The dominant kernel is the region-phase sweep
kernel; its roofline line uses the algorithmic bytes of a sweep
(2 b_q N_q + 2 b_x H W) over the HIP-event-timed kernel durations.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def workload(name):
    if name == "c3":
        return dict(workload="dykstra_1024sq_sides1-16_fp32", H=1024, W=1024, n_e=2000,
                    sides=list(range(1, 17)), dtype="fp32", tol=1e-5, max_sweeps=5000,
                    inc="f32")
    if name == "c3bf16":
        return dict(workload="dykstra_1024sq_sides1-16_fp32_bf16inc", H=1024, W=1024, n_e=2000,
                    sides=list(range(1, 17)), dtype="fp32", tol=1e-5, max_sweeps=5000,
                    inc="bf16")
    if name == "c2":
        return dict(workload="dykstra_512sq_sides1-8_fp32", H=512, W=512, n_e=200,
                    sides=list(range(1, 9)), dtype="fp32", tol=1e-5, max_sweeps=5000,
                    inc="f32")
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(x0, sides, r2, budget_s=15.0):
    """The FP64 oracle, as it is, on a bounded sample: a 256x256 crop of the
    same image with the same windows, whole sweeps until ~budget_s elapse."""
    import oracle
    crop = np.ascontiguousarray(x0[:256, :256], dtype=np.float64)
    nwin = oracle.window_count(256, 256, sides)
    t0 = time.perf_counter()
    _, sw, _ = oracle.dykstra(crop, sides, r2, tol=0, max_sweeps=1, order=oracle.ORDER_REGION,
                              region=16)
    one = time.perf_counter() - t0
    n = max(1, min(200, int(budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    _, sw, _ = oracle.dykstra(crop, sides, r2, tol=0, max_sweeps=n, order=oracle.ORDER_REGION,
                              region=16)
    el = time.perf_counter() - t0
    return {"value": nwin * sw / el, "unit": "window projections/s", "cores": 1,
            "kind": "oracle",
            "sample": f"256x256 crop, sides {sides[0]}..{sides[-1]}, {sw} FP64 sweeps, "
                      f"{el:.1f} s, single thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--region", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the projection of one image does not shard "
              "(see the design notes); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1503_03492_amd as smre
    import smre_inputs as gi

    wl = workload(args.workload)
    H, W, sides = wl["H"], wl["W"], wl["sides"]
    x0 = gi.emitters(H, W, n_e=wl["n_e"], seed=0).astype(np.float32)
    r2 = smre.chi2_bounds(sides)
    dev = torch.device("cuda:0")
    x0_dev = torch.from_numpy(x0).to(dev)
    x = torch.empty_like(x0_dev)
    ctx = smre.Context(0)
    ctx.set_timing(True)
    opts = smre.ProjectOptions(tol=wl["tol"], max_sweeps=wl["max_sweeps"], check_every=1,
                               region=args.region, kahan=True, guard_rel=1e-5,
                               inc=smre.INC_BF16 if wl["inc"] == "bf16" else smre.INC_SAME)

    def step():
        x.copy_(x0_dev)
        rc, rep = ctx.project(x, sides, r2, opts)
        return rc, rep

    for i in range(args.warmup):
        rc, rep = step()
        print(f"warmup {i}: {rep['sweeps']} sweeps, {rep['elapsed_ms']:.1f} ms", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc, rep = step()
        reps.append(rep)
        print(f"step: {rep['sweeps']} sweeps, {rep['elapsed_ms']:.1f} ms", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    wp = sum(r["window_projections"] for r in reps)
    sweeps = [r["sweeps"] for r in reps]
    kms = sum(r["kernel_ms"] for r in reps)
    launches = sum(r["kernel_launches"] for r in reps)
    bytes_alg = sum(r["bytes_moved"] for r in reps)
    achieved = bytes_alg / (kms * 1e-3) / 1e9 if kms > 0 else None
    out = {
        "metric": "window projections/s (full Dykstra to tol, 1024^2 image)",
        "value": wp / el,
        "unit": "window projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["workload"], "H": H, "W": W, "sides": f"1..{sides[-1]}",
                   "tol": wl["tol"], "increments": wl["inc"], "region": reps[0]["region"]},
        "time_to_tol_ms": el / args.steps * 1e3,
        "sweeps_to_tol": sweeps,
        "converged": all(r["converged"] for r in reps),
        "max_violation": max(r["max_violation"] for r in reps),
        "sweep_kernel_avg_us": kms / launches * 1e3 if launches else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": None,
                     "kernel": "region_phase",
                     "bytes_per_launch": bytes_alg / launches if launches else None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(x0.astype(np.float64), sides, r2)
        out["cpu_baseline"]["vs_gpu"] = out["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
