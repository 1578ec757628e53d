"""Benchmark: rigorous enclosure of min f for the separable multimodal workload
(f = sum a_i (x_i - c_i)^2 + b_i (1 - cos(2 pi k_i (x_i - c_i))), n = 100,
[-5, 5]^100, enclosure width 1e-6, seeded coefficients), on one MI355X.

One step = one whole solve (every sweep of the hot path until GUB - GLB <= 1e-6),
so ms_per_step is the time-to-enclosure and value is boxes bounded per second.
Prints one JSON line.  The headline uses incremental child bounds (the default);
the same workload also runs with full bounds and with the FP32 filter.  Each
roofline is that of the dominant kernel, timed with HIP events inside the library
on the solve's stream.  The CPU oracle's rate is taken on a bounded prefix of the
same workload.

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
# separable cosine, F of one term alone (no gradient): interval D, Y, sqr, scalings, 1 - C,
# sum (14) + two point evaluations of cos/sin (126) + extremum tests (2)
TERM_OPS_PER_COORD = 142


def incremental_ops_per_sweep(n: int, m: int) -> float:
    """Algorithmic FP64 operations of one sweep with incremental bounds (separable cosine):
    the n - m shared terms (F and the midpoint bound), both halves of the m split
    coordinates (F, G and the midpoint bound), and per child m interval additions for F
    (2 ops) and m additions for the midpoint bound (1 op)."""
    return (n - m) * (TERM_OPS_PER_COORD + MID_OPS_PER_COORD) + 2 * m * (BOX_OPS_PER_COORD + MID_OPS_PER_COORD) \
        + (1 << m) * m * 3


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64"])
    ap.add_argument("--cpu-sweeps", type=int, default=30, help="oracle prefix for the CPU baseline (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=128, help="requests in the serving trace (0 = skip)")
    ap.add_argument("--fp32-steps", type=int, default=5, help="solves of the same workload with the FP32 filter (0 = skip)")
    ap.add_argument("--full-steps", type=int, default=5, help="solves of the same workload with full bounds (0 = skip)")
    ap.add_argument("--workloads", type=int, default=1, help="1: also solve the n = 2, 1000 and 10000 workloads once")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2
    if args.copy_probe > 0:
        return copy_probe(args.copy_probe)

    import numpy as np
    import torch
    import paper_2507_01770_amd as ibb
    from paper_2507_01770_amd import problems as PR

    p = PR.config(1)

    def timed(steps, warmup, **kw):
        # the timed solves run without profiling; one more solve with the library's
        # kernel timers (HIP events on its stream) follows, outside the timed region
        for _ in range(warmup):
            ibb.minimize(p, fetch_boxes=False, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = [ibb.minimize(p, fetch_boxes=False, **kw) for _ in range(steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rp = ibb.minimize(p, fetch_boxes=False, profile=True, **kw)
        for r in rs + [rp]:
            assert r.status == ibb.OK and r.f_lo <= 0.0 <= r.f_hi and r.f_hi - r.f_lo <= 1e-6, (r.f_lo, r.f_hi)
            assert r.sweeps == rp.sweeps and r.boxes_evaluated == rp.boxes_evaluated
        return rs + [rp], dt

    # headline: incremental child bounds (the default)
    phase("headline: incremental bounds")
    res, dt = timed(args.steps, args.warmup)
    boxes = sum(r.boxes_evaluated for r in res[:-1])
    r0 = res[-1]
    # dominant kernel: the persistent sweep kernel (selection and the children's bounds in
    # one workgroup, up to 256 sweeps per launch); one unit of work is one sweep
    ib_ops_sweep = incremental_ops_per_sweep(p.n, min(p.n, 10))
    n_sw = max(1, r0.n_select_launches)
    t_sweep = r0.t_select_ms * 1e-3 / n_sw
    ach = ib_ops_sweep / t_sweep / 1e12 if t_sweep > 0 else 0.0
    roofline = {
        "bound": "alu", "kernel": "k_sweeps_ib<SEP_COS> (persistent, one workgroup)", "per": "sweep",
        "achieved": round(ach, 6), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 8),
        "traffic": measured_traffic(), "avg_sweep_us": round(t_sweep * 1e6, 3), "sweeps_per_solve": r0.sweeps,
        "flops_per_sweep": round(ib_ops_sweep),
    }

    # the same workload with full bounds (every child over all n terms): k_bound's roofline
    full = None
    if args.full_steps > 0:
        phase("full bounds")
        rf, df = timed(args.full_steps, 1, incremental=False)
        q = rf[-1]
        formed = q.boxes_evaluated - 1          # children (the root is bounded by another kernel)
        ops = p.n * (formed * BOX_OPS_PER_COORD + (q.ub_evaluated - 1) * MID_OPS_PER_COORD) * 1.0
        tb = q.t_bound_ms * 1e-3
        a = ops / tb / 1e12 if tb > 0 else 0.0
        full = {"boxes_per_s": round(sum(r.boxes_evaluated for r in rf[:-1]) / df, 1),
                "ms_per_solve": round(df / args.full_steps * 1e3, 4), "sweeps": q.sweeps,
                "bound_shape": q.bound_shape,
                "roofline": {"bound": "alu", "kernel": "k_bound<SEP_COS>", "achieved": round(a, 4),
                             "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": round(a / PEAK_FP64_TFLOPS, 5),
                             "avg_launch_us": round(q.t_bound_ms * 1e3 / max(1, q.n_bound_launches), 3),
                             "flops_per_launch": round(ops / max(1, q.n_bound_launches))},
                "select_avg_launch_us": round(q.t_select_ms * 1e3 / max(1, q.n_select_launches), 3)}

    fp32 = None
    if args.fp32_steps > 0:
        phase("fp32 filter")
        r32, d32 = timed(args.fp32_steps, 1, precision="fp32_bulk")
        q = r32[-1]
        fp32 = {"boxes_per_s": round(sum(r.boxes_evaluated for r in r32[:-1]) / d32, 1),
                "ms_per_solve": round(d32 / args.fp32_steps * 1e3, 4),
                "sweeps": q.sweeps, "boxes_per_solve": q.boxes_evaluated,
                "fp32_pruned": q.fp32_pruned, "fp64_confirmed": q.fp64_confirmed, "fp32_sweeps": q.fp32_sweeps,
                "bound_avg_launch_us": round(q.t_bound_ms * 1e3 / max(1, q.n_bound_launches), 3),
                "enclosure": [q.f_lo, q.f_hi]}

    # the other workloads, solved completely once each (incremental bounds)
    workloads = None
    if args.workloads:
        phase("other workloads")
        workloads = {}
        for cfg in (0, 2, 3):
            phase(f"workload {cfg}")
            q = PR.config(cfg)
            if cfg != 3:
                ibb.minimize(q, fetch_boxes=False)
            torch.cuda.synchronize()
            tq = time.perf_counter()
            rq = ibb.minimize(q, fetch_boxes=False)
            torch.cuda.synchronize()
            dq = time.perf_counter() - tq
            assert rq.status == ibb.OK and rq.f_lo <= 0.0 <= rq.f_hi and rq.f_hi - rq.f_lo <= 1e-6, (cfg, rq.f_lo, rq.f_hi)
            workloads[f"{PR.FAMILY_NAMES[q.family]}_n{q.n}"] = {
                "time_to_enclosure_ms": round(dq * 1e3, 3), "sweeps": rq.sweeps, "boxes": rq.boxes_evaluated,
                "boxes_per_s": round(rq.boxes_evaluated / dq, 1), "enclosure": [rq.f_lo, rq.f_hi]}

    if args.serve_requests > 0:
        phase("serving")
    serving = serve_bench(args.serve_requests) if args.serve_requests > 0 else None

    # the CPU oracle last, after all GPU work
    cpu = None
    if args.cpu_sweeps > 0:
        phase("cpu baseline (oracle)")
        from oracle import oracle as O
        tc = time.perf_counter()
        o = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6, max_sweeps=args.cpu_sweeps, incremental=True)
        tcpu = time.perf_counter() - tc
        cpu = {"value": round(o.boxes_evaluated / tcpu, 2), "unit": "boxes/s", "cores": 1, "kind": "oracle",
               "sample": f"first {o.sweeps} sweeps of the same workload with incremental child bounds "
                         f"({o.boxes_evaluated} boxes, {tcpu:.1f} s, single thread, fesetround per endpoint operation)"}

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
            "time_to_enclosure_ms": round(float(np.median([r.seconds for r in res[:-1]])) * 1e3, 4),
            "sweeps": r0.sweeps, "boxes_per_solve": r0.boxes_evaluated,
            "enclosure": [r0.f_lo, r0.f_hi], "bounds": "incremental",
            "full_bounds": full,
            "fp32_bulk_full_bounds": fp32,
            "other_workloads": workloads,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)
    return 0


def phase(name: str) -> None:
    """A progress line on stderr (the JSON result line goes to stdout)."""
    print(f"bench: {name}", file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per sweep of the persistent sweep kernel, from the committed rocprofv3 FETCH_SIZE and
    WRITE_SIZE counts (scaled by a plain copy's), when the kernel sources are the ones measured; else None."""
    import glob
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_bytes_sep_cos_n100.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(\{.*?\})\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    src = sorted(glob.glob(os.path.join(ROOT, "paper_2507_01770_amd", "csrc", "*")))
    h = hashlib.sha256(b"".join(open(f, "rb").read() for f in src)).hexdigest()[:16]
    return rec["bytes_per_sweep"] if rec.get("source_hash") == h else None


def copy_probe(mib: int) -> int:
    """A plain device-to-device copy of `mib` MiB, for scaling the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4}), flush=True)
    return 0


SERVE_MAX_SWEEPS = 500     # per-request sweep budget (some chained requests do not converge quickly)


def serve_bench(count: int) -> dict:
    """Serving workload: `count` requests (n log-uniform in [2, 2000], family uniform over the
    three, seeded coefficients), enclosure width 1e-6, at most SERVE_MAX_SWEEPS sweeps each.
    1) closed loop: all requests submitted at once -> capacity mu (problems/s);
    2) Poisson arrivals at 0.8 mu through the continuous-batching server -> problems/s, p50/p99
       of completion - arrival;
    3) the same arrivals served one at a time, FIFO, by ibb_solve (plain FP64, no batching)."""
    import numpy as np
    import paper_2507_01770_amd as ibb
    from paper_2507_01770_amd import problems as PR

    reqs = PR.serving_trace(count=count, seed=105, rate=1.0)
    probs = [p for _, p in reqs]
    gaps = np.array([t for t, _ in reqs])
    gaps = np.diff(np.concatenate([[0.0], gaps]))          # unit-rate exponential gaps

    def run_server(arrivals):
        with ibb.Server(mem_budget_bytes=64 << 30, max_slots=64) as srv:
            t0 = time.perf_counter()
            tickets, t_arr, done = [], [], {}
            i = 0
            while len(done) < len(probs):
                now = time.perf_counter() - t0
                while i < len(probs) and arrivals[i] <= now:
                    tickets.append(srv.submit(probs[i], max_sweeps=SERVE_MAX_SWEEPS))
                    t_arr.append(arrivals[i])
                    i += 1
                for k, t in enumerate(tickets):
                    if t not in done:
                        r = srv.poll(t)
                        if r is not None:
                            done[t] = (time.perf_counter() - t0, r.status)
                time.sleep(0.0002)
            st = srv.stats()
        lat = np.array([done[t][0] - a for t, a in zip(tickets, t_arr)])
        makespan = max(v[0] for v in done.values()) - arrivals[0]
        ok = sum(v[1] == ibb.OK for v in done.values())
        return lat, makespan, ok, st

    lat0, span0, ok0, st0 = run_server(np.zeros(len(probs)))
    mu = len(probs) / span0
    lam = 0.8 * mu
    arrivals = np.cumsum(gaps) / lam
    lat, span, ok, st = run_server(arrivals)
    # one at a time, FIFO, same arrivals
    t0 = time.perf_counter()
    free_at, lat1 = 0.0, []
    for a, p in zip(arrivals, probs):
        start = max(a, free_at)
        while time.perf_counter() - t0 < start:
            time.sleep(0.0002)
        ibb.minimize(p, max_sweeps=SERVE_MAX_SWEEPS, fetch_boxes=False)
        free_at = time.perf_counter() - t0
        lat1.append(free_at - a)
    lat1 = np.array(lat1)
    span1 = free_at - arrivals[0]
    return {
        "requests": len(probs), "max_sweeps_per_request": SERVE_MAX_SWEEPS, "converged": int(ok),
        "capacity_problems_per_s": round(mu, 2), "arrival_rate": round(lam, 2),
        "problems_per_s": round(len(probs) / span, 2),
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2), "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
        "max_concurrent": st["max_active"],
        "one_at_a_time": {"problems_per_s": round(len(probs) / span1, 2),
                          "p50_ms": round(float(np.percentile(lat1, 50)) * 1e3, 2),
                          "p99_ms": round(float(np.percentile(lat1, 99)) * 1e3, 2)},
    }


if __name__ == "__main__":
    sys.exit(main())
