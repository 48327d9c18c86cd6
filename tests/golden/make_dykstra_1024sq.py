"""Write the FP64 oracle's projection of the 1024 x 1024 emitter image.

Input: smre_inputs.emitters(1024, 1024, n_e=2000, seed=0) rounded to float32
(the FP32 library path reads that image; the oracle gets the same values in
double).  Family: every window of sides 1..16 fully inside the image, bounds
the chi-square(s^2) 0.9 quantiles.  Order: the region order with R = 16
(Sec. 2.3 leaves the order of overlapping sets open; the limit does not depend
on it).  Stopping rule: max |x - x_prev| < tol between sweep ends, checked
every sweep -- the rule of the FP32 headline run.

Stages: tol 1e-5 from zero increments (the headline stopping point), then the
same Dykstra continued from those increments (x = x0 - sum_S I_S) to tol 1e-6
and 1e-7, closer to the exact projection.  Each stage is saved as soon as it
ends, with its sweep count, last change, feasibility and wall time.

Only oracle/ computes anything here.  Needs ~26 GB of memory (two FP64
increment sets of 1496 x 1024 x 1024) and hours of CPU:
    python tests/golden/make_dykstra_1024sq.py [--threads N]
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import smre_inputs as gi  # noqa: E402

OUT = os.path.join(HERE, "dykstra_1024sq_sides1-16_r16.npz")
SIDES = list(range(1, 17))
REGION = 16


def input_image():
    return gi.emitters(1024, 1024, n_e=2000, seed=0).astype(np.float32)


def input_sha256(x32):
    return hashlib.sha256(np.ascontiguousarray(x32, dtype=np.float32).tobytes()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--tols", default="1e-5,1e-6,1e-7")
    ap.add_argument("--max-sweeps", type=int, default=20000)
    a = ap.parse_args()
    x32 = input_image()
    x0 = x32.astype(np.float64)
    r2 = oracle.chi2_bounds(SIDES)
    nt = oracle.set_threads(a.threads)
    out = {"input_sha256": np.array(input_sha256(x32)), "sides": np.array(SIDES, np.int32),
           "radius2": r2, "region": np.array(REGION), "threads": np.array(nt),
           "cpu": np.array(_cpu_model())}
    incs = None
    total = 0
    for k, tol in enumerate(float(t) for t in a.tols.split(",")):
        t0 = time.time()
        if incs is None:
            z, sw, d, incs = oracle.dykstra(x0, SIDES, r2, tol=tol, max_sweeps=a.max_sweeps,
                                            order=oracle.ORDER_REGION, region=REGION,
                                            want_incs=True)
        else:
            z, sw, d = oracle.dykstra(x0, SIDES, r2, tol=tol, max_sweeps=a.max_sweeps,
                                      order=oracle.ORDER_REGION, region=REGION, incs0=incs,
                                      in_place=True)
        el = time.time() - t0
        total += sw
        viol = oracle.max_violation(z, SIDES, r2)
        tag = f"{tol:.0e}"
        out[f"z_tol{tag}"] = z
        out[f"sweeps_tol{tag}"] = np.array(total)
        out[f"delta_tol{tag}"] = np.array(d)
        out[f"violation_tol{tag}"] = np.array(viol)
        out[f"seconds_tol{tag}"] = np.array(el)
        np.savez_compressed(OUT + ".tmp.npz", **out)
        os.replace(OUT + ".tmp.npz", OUT)
        print(f"tol {tol:g}: {total} sweeps in all (+{sw} in {el:.0f} s, {nt} threads), "
              f"last change {d:.3e}, max violation {viol:.3e}", flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
