"""Benchmark: rigorous enclosure of min f for the separable multimodal workload
(f = sum a_i (x_i - c_i)^2 + b_i (1 - cos(2 pi k_i (x_i - c_i))), n = 100,
[-5, 5]^100, enclosure width 1e-6, seeded coefficients), on one MI355X.

One step = one whole solve (every sweep of the hot path until GUB - GLB <= 1e-6),
so ms_per_step is the time-to-enclosure and value is boxes bounded per second.
Prints one JSON line.  Also reports the roofline of the dominant kernel
(k_bound, timed with HIP events inside the library on the solve's stream) and
the CPU oracle's rate on a bounded prefix of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 operations per child per coordinate (adds and muls count 1,
# fma 2), counted from the expression trees of the separable cosine family:
#   box pass (F and G): interval D, Y, sqr, scalings, sums, gradient product
#   (46 ops) plus two point evaluations of cos/sin(2 pi y) at the endpoints of Y
#   (63 ops each: reduction 3, split squares 3, sine 2-term head 9 + tail 16 +
#   corrections 10 + enclosure 5, cosine head 5 + tail 16 + corrections 7 +
#   enclosure 5, and 2 for the extremum tests) -> 172
#   midpoint pass (upper bound): midpoint 2, D/Y/sqr/scalings/sum of the upper
#   endpoints 14, two point evaluations 126 -> 142
BOX_OPS_PER_COORD = 172
MID_OPS_PER_COORD = 142
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 64 lanes x 2 (fma) x 2.4 GHz


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64"])
    ap.add_argument("--cpu-sweeps", type=int, default=30, help="oracle prefix for the CPU baseline (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import paper_2507_01770_amd as ibb
    from paper_2507_01770_amd import problems as PR

    p = PR.config(1)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        ibb.minimize(p, fetch_boxes=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [ibb.minimize(p, fetch_boxes=False, profile=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    boxes = sum(r.boxes_evaluated for r in res)
    for r in res:
        assert r.status == ibb.OK and r.f_lo <= 0.0 <= r.f_hi and r.f_hi - r.f_lo <= 1e-6, (r.f_lo, r.f_hi)

    # roofline of k_bound: algorithmic FP64 ops over the summed kernel time
    r0 = res[-1]
    formed = r0.boxes_evaluated - 1          # children (the root is bounded by another kernel)
    ub_children = r0.ub_evaluated - 1
    ops = p.n * (formed * BOX_OPS_PER_COORD + ub_children * MID_OPS_PER_COORD) * 1.0
    t_bound = r0.t_bound_ms * 1e-3
    achieved = ops / t_bound / 1e12 if t_bound > 0 else 0.0
    roofline = {
        "bound": "alu", "kernel": "k_bound<SEP_COS>", "achieved": round(achieved, 4), "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 5), "traffic": None,
        "avg_launch_us": round(r0.t_bound_ms * 1e3 / max(1, r0.n_bound_launches), 3),
        "launches_per_solve": r0.n_bound_launches,
        "flops_per_launch": round(ops / max(1, r0.n_bound_launches)),
        "select_avg_launch_us": round(r0.t_select_ms * 1e3 / max(1, r0.n_select_launches), 3),
    }

    cpu = None
    if args.cpu_sweeps > 0:
        from oracle import oracle as O
        tc = time.perf_counter()
        o = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6, max_sweeps=args.cpu_sweeps)
        tcpu = time.perf_counter() - tc
        cpu = {"value": round(o.boxes_evaluated / tcpu, 2), "unit": "boxes/s", "cores": 1, "kind": "oracle",
               "sample": f"first {o.sweeps} sweeps of the same workload ({o.boxes_evaluated} boxes, {tcpu:.1f} s, "
                         f"single thread, fesetround per endpoint operation)"}

    line = {
        "metric": "boxes/sec and time-to-enclosure (width 1e-6); served problems/sec + p50/p99",
        "value": round(boxes / dt, 1),
        "unit": "boxes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "separable cosine family, n=100, domain [-5,5]^100, enclosure width 1e-6, seed 102",
            "precision": args.precision, "select_k": 1, "split_dims": 10,
            "time_to_enclosure_ms": round(float(np.median([r.seconds for r in res])) * 1e3, 4),
            "sweeps": r0.sweeps, "boxes_per_solve": r0.boxes_evaluated,
            "enclosure": [r0.f_lo, r0.f_hi],
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
