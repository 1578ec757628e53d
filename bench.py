"""Benchmark on one MI355X: rigorous enclosure of min f at width 1e-6.

Headline (the largest single-GPU workload): the non-smooth separable family
f = sum s_i |x_i - c_i| + b_i sin^2(pi k_i (x_i - c_i)), n = 10,000, domain
[-10, 10]^10000, seeded coefficients, enclosure width 1e-6, one box per sweep as
in the paper with incremental child bounds and the term cache, each sweep on
several workgroups (selection, row and base terms over coordinate blocks, slot
sums, children).  One step = one whole solve, so ms_per_step is the time to enclosure
and value is boxes bounded per second.

Also measured in the same run (extra keys of the JSON line):
  * the separable cosine family at n = 100: one box per sweep (persistent
    kernel), and K = 32 boxes per sweep (the paper's one-region selection
    widened so that one sweep fills the chip: K = ceil(2^16 / (2^m ceil(n/64)))),
    in plain FP64 with full bounds, with the FP32 filter, and with incremental
    bounds; the roofline of the full-bounds kernel at that occupancy;
  * the other workloads (n = 2 and the chained n = 1000), solved once each;
  * serving: the 4096-request trace through the continuous-batching server
    (closed loop -> capacity mu, then Poisson arrivals at 0.8 mu), and on its
    first requests the same arrivals served one at a time by plain FP64 solves
    (full bounds, one kernel launch per step);
  * the paper's own experiments (Sec. 4 schedule, n = 50, the benchmark functions
    of SI Appendix A as expression tapes): time, iterations and output regions
    per function, beside the paper's cloud-server times (other hardware);
  * the CPU oracle bounding children of the headline workload's first sweep (its
    per-child work), on one host thread and as one copy per host core.
The headline's roofline is per sweep and against HBM: with the term cache a sweep at
n = 10,000 mostly moves bytes (the live keys' lower bounds scanned, the selected
row built, the parent's cached terms read and the box's written; cached_sweep_bytes).
Other rooflines use the algorithmic operation counts per child and coordinate (F, its
gradient and the midpoint bound; one directed endpoint operation = 1 op):
about 175 for the separable families (five sin/cos point evaluations of about 25
operations each and about 50 interval endpoint operations), 64 for the chained
family, over each kernel's average launch time measured with HIP events on the
stream it runs on.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SEP_OPS = 175     # algorithmic operations per child and coordinate, separable families
CHAIN_OPS = 64    # the chained family
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 64 lanes x 2 (fma) x 2.4 GHz
# the paper's times at n = 50 on its cloud server (one GPU; Tables S2-S10 and Table 2,
# last column), for context: other hardware, another implementation
PAPER_CLOUD_S50 = {"ackley": 11, "belegundu": 6, "breiman": 5, "fu": 13, "griewank": 9, "levy": 15,
                   "rastrigin": 6, "salomon": 5, "styblinski": 7, "zabinsky": 9}


def incremental_ops_per_sweep(n: int, m: int, per_coord: int = SEP_OPS) -> float:
    """Algorithmic operations of one incremental sweep: the n - m shared terms and
    both halves of the m split coordinates (n + m coordinate evaluations), then per
    child m interval additions for F (2 ops) and m for the midpoint bound (1 op)."""
    return (n + m) * per_coord + (1 << m) * m * 3


def cached_sweep_bytes(n: int, keys: float) -> float:
    """HBM bytes of one sweep with the term cache (n >= 1024): the selection's scan of
    the live keys' lower bounds (8 B each), the selected box's row built from its
    parent's (16 n read, 16 n written), the parent's cached terms read and the box's
    own written (24 n each)."""
    return 8.0 * keys + 80.0 * n


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-boxes", type=int, default=256,
                    help="children of the headline workload bounded by the oracle for the CPU baseline (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=4096, help="requests in the serving trace (0 = skip)")
    ap.add_argument("--serve-max-sweeps", type=int, default=8000,
                    help="sweep budget of each serving request (requests that reach it are counted apart)")
    ap.add_argument("--serve-compare", type=int, default=96,
                    help="first requests of the trace also served one at a time by plain FP64 solves")
    ap.add_argument("--k-steps", type=int, default=3, help="solves per form of the n = 100 workload (0 = skip)")
    ap.add_argument("--workloads", type=int, default=1, help="1: also solve the n = 2 and chained n = 1000 workloads")
    ap.add_argument("--headline", type=int, default=1, help="0: skip the headline solves (profiling runs)")
    ap.add_argument("--paper-n", type=int, default=50,
                    help="n of the paper's benchmark-function experiments (Sec. 4 schedule; 0 = skip)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2
    if args.copy_probe > 0:
        return copy_probe(args.copy_probe)

    import numpy as np
    import torch
    import paper_2507_01770_amd as ibb
    from paper_2507_01770_amd import problems as PR

    def timed(p, steps, warmup, **kw):
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
        return rs, rp, dt

    # ---- headline: workload 3 (n = 10,000), one box per sweep, each on several workgroups
    p3 = PR.config(3)
    head = roofline = None
    if args.headline:
        phase("headline: non-smooth separable n = 10000")
        rs, rp, dt = timed(p3, args.steps, args.warmup)
        m = min(p3.n, 10)
        # one sweep is five launches on the library's stream (k_select_part on long
        # lists, k_ib_pick, k_ib_rowterms, k_ib_slots, k_ib_finish), timed together by
        # its HIP events around them; with the term cache a sweep moves bytes rather
        # than evaluating terms, so it is priced against HBM, the keys scanned per
        # sweep being the sweeps' live counts
        sweeps = max(1, rp.n_select_launches)
        t_sweep = rp.t_select_ms * 1e-3 / sweeps
        keys = float(np.mean(rp.trace_nlive)) if rp.trace_nlive.size else 0.0
        bytes_sweep = cached_sweep_bytes(p3.n, keys)
        ach = bytes_sweep / t_sweep / 1e9 if t_sweep > 0 else 0.0
        ops_sweep = 3 * m * SEP_OPS + 3 * p3.n + (1 << m) * m * 3   # fresh terms, the base sum, the children
        roofline = {
            "bound": "hbm",
            "kernel": "one sweep: k_select_part, k_ib_pick<512>, k_ib_rowterms<SEP_ABS_SIN2>, k_ib_slots, "
                      "k_ib_finish<512, SEP_ABS_SIN2> (per sweep; achieved and traffic per sweep)",
            "achieved": round(ach, 3), "peak": 8000.0, "unit": "GB/s", "frac": round(ach / 8000.0, 6),
            "traffic": measured_traffic(), "avg_sweep_us": round(t_sweep * 1e6, 3), "sweeps_timed": sweeps,
            "bytes_per_sweep": round(bytes_sweep), "mean_live_keys": round(keys),
            "alu_tflops": round(ops_sweep / t_sweep / 1e12, 6) if t_sweep > 0 else 0.0,
            "ops_per_sweep": ops_sweep,
        }
        head = {"rs": rs, "rp": rp, "dt": dt}

    # ---- workload 1 (n = 100): K = 1 persistent; K = 32 full bounds FP64 / FP32 filter / incremental
    forms = None
    if args.k_steps > 0:
        p1 = PR.config(1)
        m1 = min(p1.n, 10)
        K = -(-(1 << 16) // ((1 << m1) * (-(-p1.n // 64))))
        forms = {"workload": "separable cosine family, n=100, [-5,5]^100, width 1e-6, seed 102", "K": K}
        for name, kw in (("k1_incremental", dict()),
                         ("kK_full_fp64", dict(select_k=K, incremental=False)),
                         ("kK_full_fp32_bulk", dict(select_k=K, precision="fp32_bulk")),
                         ("kK_incremental", dict(select_k=K, incremental=True))):
            phase(f"n = 100: {name}")
            rs1, rp1, dt1 = timed(p1, args.k_steps, 1, **kw)
            d = {"boxes_per_s": round(sum(r.boxes_evaluated for r in rs1) / dt1, 1),
                 "ms_per_solve": round(dt1 / args.k_steps * 1e3, 4), "sweeps": rp1.sweeps,
                 "boxes_per_solve": rp1.boxes_evaluated, "enclosure": [rp1.f_lo, rp1.f_hi]}
            if rp1.n_bound_launches:
                if kw.get("incremental"):
                    # k_ib_parents: one workgroup per selected box; per box the incremental
                    # sweep's work (its 2^m children, each parent's shared terms once)
                    parents = (rp1.boxes_evaluated - 1) / (1 << m1)
                    ops = parents * incremental_ops_per_sweep(p1.n, m1)
                    kname = "k_ib_parents<512, SEP_COS>"
                else:
                    formed = rp1.boxes_evaluated - 1 - rp1.fp32_pruned   # children bounded in FP64
                    ops = p1.n * formed * SEP_OPS * 1.0
                    kname = "k_bound<SEP_COS> (shape %d)" % rp1.bound_shape
                tb = rp1.t_bound_ms * 1e-3
                a = ops / tb / 1e12 if tb > 0 else 0.0
                d["bound_kernel"] = {
                    "kernel": kname, "achieved": round(a, 4),
                    "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": round(a / PEAK_FP64_TFLOPS, 5),
                    "avg_launch_us": round(rp1.t_bound_ms * 1e3 / rp1.n_bound_launches, 3),
                    "ops_per_launch": round(ops / rp1.n_bound_launches),
                    "select_avg_launch_us": round(rp1.t_select_ms * 1e3 / max(1, rp1.n_select_launches), 3)}
            if rp1.fp32_sweeps:
                d.update(fp32_pruned=rp1.fp32_pruned, fp64_confirmed=rp1.fp64_confirmed, fp32_sweeps=rp1.fp32_sweeps)
            forms[name] = d

    # ---- the other workloads, solved once each (incremental bounds, one box per sweep)
    workloads = None
    if args.workloads:
        workloads = {}
        for cfg in (0, 2):
            phase(f"workload {cfg}")
            q = PR.config(cfg)
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

    # ---- the paper's own experiments (Sec. 4) with the generic family: n = 50, ten cycled
    # coordinates cut into four pieces (4^10 subregions per iteration), ten diagonal samples,
    # stop at width 1e-4; the paper's cloud-server times are context (other hardware)
    paper = None
    if args.paper_n > 0:
        from paper_2507_01770_amd import tapes as TP
        paper = {"n": args.paper_n, "schedule": "4 pieces x 10 cycled coordinates, 10 diagonal samples, width 1e-4"}
        for name, make in TP.PAPER_FUNCTIONS.items():
            if name == "rosenbrock":
                continue
            phase(f"paper experiment: {name} n = {args.paper_n}")
            q = make(args.paper_n)
            kw = dict(split_dims=10, pieces=4, diag_samples=10, tol_f=1e300, tol_x=1e-4, max_sweeps=100000,
                      fetch_boxes=False)
            ibb.minimize(q, **kw)
            torch.cuda.synchronize()
            tq = time.perf_counter()
            rq = ibb.minimize(q, **kw)
            torch.cuda.synchronize()
            dq = time.perf_counter() - tq
            paper[name] = {"seconds": round(dq, 3), "iterations": rq.sweeps, "regions": rq.n_boxes,
                           "boxes_per_s": round(rq.boxes_evaluated / dq, 1), "enclosure": [rq.f_lo, rq.f_hi],
                           "paper_cloud_server_s": PAPER_CLOUD_S50.get(name) if args.paper_n == 50 else None}

    serving = None
    if args.serve_requests > 0:
        phase("serving")
        serving = serve_bench(args.serve_requests, args.serve_compare, args.serve_max_sweeps)

    # ---- the CPU oracle last, after all GPU work
    cpu = None
    if args.cpu_boxes > 0:
        phase("cpu baseline (oracle)")
        cpu = cpu_baseline(p3, args.cpu_boxes)

    rs, rp, dt = (head["rs"], head["rp"], head["dt"]) if head else ([], None, 0.0)
    boxes = sum(r.boxes_evaluated for r in rs)
    line = {
        "metric": "boxes/sec and time-to-enclosure (width 1e-6); served problems/sec + p50/p99",
        "value": round(boxes / dt, 1) if dt > 0 else None,
        "unit": "boxes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4) if dt > 0 else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "non-smooth separable family, n=10000, domain [-10,10]^10000, enclosure width 1e-6, "
                        "seed 104, one box per sweep, 10 bisected coordinates",
            "time_to_enclosure_ms": round(float(np.median([r.seconds for r in rs])) * 1e3, 3) if rs else None,
            "sweeps": rp.sweeps if rp else None, "boxes_per_solve": rp.boxes_evaluated if rp else None,
            "enclosure": [rp.f_lo, rp.f_hi] if rp else None, "bounds": "incremental",
            "box_coord_per_s": round(boxes * p3.n / dt, 1) if dt > 0 else None,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "n100_forms": forms,
        "other_workloads": workloads,
        "serving": serving,
        "paper_experiments": paper,
    }
    print(json.dumps(line), flush=True)
    return 0


_T_START = time.perf_counter()


def phase(name: str) -> None:
    """A progress line on stderr (the JSON result line goes to stdout)."""
    print(f"bench: [{time.perf_counter() - _T_START:7.1f} s] {name}", file=sys.stderr, flush=True)


def first_children(p, count: int, m: int = 10):
    """The first `count` children of the workload's first sweep: the domain with its
    first m coordinates halved (child r takes the upper half of coordinate j when bit
    j of r is set), every endpoint a double of the domain's halving."""
    import numpy as np
    mid = 0.5 * p.lower + 0.5 * p.upper
    lo = np.tile(p.lower, (count, 1))
    hi = np.tile(p.upper, (count, 1))
    for r in range(count):
        for j in range(m):
            if (r >> j) & 1:
                lo[r, j] = mid[j]
            else:
                hi[r, j] = mid[j]
    return lo, hi


def cpu_baseline(p, boxes: int) -> dict:
    """The oracle bounding children of the workload's first sweep (F, the first-order
    test and the midpoint bound of each, as its solve does per child): `boxes` of them on
    one host thread, then one copy per host core at once (the oracle itself is serial)."""
    from oracle import oracle as O
    lo, hi = first_children(p, boxes)
    tc = time.perf_counter()
    O.eval_boxes(p.family, p.coef, p.lower, p.upper, lo, hi)
    t1 = time.perf_counter() - tc
    one = boxes / t1
    phase(f"cpu baseline: one thread, {boxes} boxes in {t1:.1f} s")
    cores = min(16, len(os.sched_getaffinity(0)))
    code = ("import sys, time; sys.path.insert(0, %r); import bench; from oracle import oracle as O; "
            "from paper_2507_01770_amd import problems as PR; p = PR.config(3); lo, hi = bench.first_children(p, %d); "
            "t = time.perf_counter(); O.eval_boxes(p.family, p.coef, p.lower, p.upper, lo, hi); "
            "print('bench: cpu baseline: a copy finished in %%.1f s' %% (time.perf_counter() - t), "
            "file=sys.stderr, flush=True)") % (ROOT, boxes)
    tc = time.perf_counter()
    procs = [subprocess.Popen([sys.executable, "-c", code]) for _ in range(cores)]
    ok = all(pr.wait() == 0 for pr in procs)
    tall = time.perf_counter() - tc
    return {"value": round(one, 2), "unit": "boxes/s", "cores": 1, "kind": "oracle",
            "sample": f"{boxes} children of the headline workload's first sweep bounded by the oracle "
                      f"(F, first-order test, midpoint bound: its per-child work), {t1:.1f} s on one thread, "
                      f"rounding mode switched per endpoint operation",
            "all_cores": {"value": round(cores * boxes / tall, 2) if ok else None, "unit": "boxes/s",
                          "cores": cores, "sample": f"{cores} copies of the same sample at once, {tall:.1f} s"},
            "host_cpus": os.cpu_count()}


def measured_traffic():
    """HBM bytes per sweep of the headline (its five launches), from the committed
    rocprofv3 FETCH_SIZE and WRITE_SIZE counts (scaled by a plain copy's), when the kernel
    sources are the ones measured; else None."""
    import glob
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_bytes_sep_abs_sin2_n10000.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(\{.*?\})\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    return rec["bytes_per_sweep"] if rec.get("source_hash") == kernel_source_hash() else None


def kernel_source_hash() -> str:
    import glob
    import hashlib
    src = sorted(glob.glob(os.path.join(ROOT, "paper_2507_01770_amd", "csrc", "*")))
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in src)).hexdigest()[:16]


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


def serve_bench(count: int, compare: int, max_sweeps: int) -> dict:
    """Serving workload: `count` requests (n log-uniform in [2, 2000], family uniform over the
    three, seeded coefficients), each enclosed to width 1e-6 within `max_sweeps` sweeps.
    1) closed loop: the first 512 requests submitted at once -> capacity mu (problems/s);
    2) Poisson arrivals of all requests at 0.8 mu through the continuous-batching server ->
       problems/s, p50/p99 of completion - arrival (converged and budget-stopped requests
       counted apart);
    3) on the first `compare` requests, the same arrivals through the server and served one at
       a time, FIFO, by ibb_solve in plain FP64 (full bounds, a selection and a bound kernel
       launch per sweep, no batching, no persistent kernel).
    The server holds at most 96 GiB of box lists: a request whose list would grow past that
    ends early, not converged (stop reason 8), as after its sweep budget (stop reason 2)."""
    import numpy as np
    import paper_2507_01770_amd as ibb
    from paper_2507_01770_amd import problems as PR

    reqs = PR.serving_trace(count=count, seed=105, rate=1.0)
    probs = [p for _, p in reqs]
    gaps = np.array([t for t, _ in reqs])
    gaps = np.diff(np.concatenate([[0.0], gaps]))          # unit-rate exponential gaps

    def run_server(ps, arrivals):
        with ibb.Server(mem_budget_bytes=96 << 30, max_slots=256) as srv:
            t0 = time.perf_counter()
            tickets, t_arr, done = [], [], {}
            pending = []
            i = 0
            t_note = t0
            while len(done) < len(ps):
                now = time.perf_counter() - t0
                while i < len(ps) and arrivals[i] <= now:
                    t = srv.submit(ps[i], max_sweeps=max_sweeps)
                    tickets.append(t)
                    pending.append(t)
                    t_arr.append(arrivals[i])
                    i += 1
                still = []
                for t in pending:
                    try:
                        r = srv.poll(t)
                        if r is None:
                            still.append(t)
                            continue
                        done[t] = (time.perf_counter() - t0, r.status, r.stop_reason)
                    except ibb.IbbError as e:   # this request only (its result could not be formed)
                        done[t] = (time.perf_counter() - t0, -1, str(e))
                pending = still
                if time.perf_counter() - t_note > 20.0:
                    t_note = time.perf_counter()
                    phase(f"serving: {len(done)} of {len(ps)} requests done, {len(pending)} in flight")
                time.sleep(0.0002)
            st = srv.stats()
        lat = np.array([done[t][0] - a for t, a in zip(tickets, t_arr)])
        conv = np.array([done[t][1] == ibb.OK for t in tickets])
        makespan = max(v[0] for v in done.values()) - arrivals[0]
        st["stops"] = {"converged": int(conv.sum()),
                       "sweep_budget": sum(v[1] == ibb.NOT_CONVERGED and v[2] == 2 for v in done.values()),
                       "memory_budget": sum(v[1] == ibb.NOT_CONVERGED and v[2] == 8 for v in done.values()),
                       "errors": sum(v[1] == -1 for v in done.values())}
        return lat, conv, makespan, st

    def pct(a, q):
        return round(float(np.percentile(a, q)) * 1e3, 2) if len(a) else None

    head = probs[:512]
    phase(f"serving: closed loop, the first {len(head)} requests")
    lat0, conv0, span0, st0 = run_server(head, np.zeros(len(head)))
    mu = len(head) / span0
    lam = 0.8 * mu
    arrivals = np.cumsum(gaps) / lam
    phase(f"serving: Poisson arrivals at {lam:.1f}/s")
    lat, conv, span, st = run_server(probs, arrivals)
    out = {
        "requests": len(probs), "converged": int(conv.sum()),
        "capacity_problems_per_s": round(mu, 2), "capacity_sample_requests": len(head), "arrival_rate": round(lam, 2),
        "problems_per_s": round(len(probs) / span, 2),
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
        "p50_ms_converged": pct(lat[conv], 50), "p99_ms_converged": pct(lat[conv], 99),
        "max_concurrent": st["max_active"], "stops": st["stops"], "max_sweeps_per_request": max_sweeps,
    }
    if compare > 0:
        ps = probs[:compare]
        arr = arrivals[:compare] - arrivals[0]
        phase(f"serving: first {compare} requests through the server")
        latc, convc, spanc, _ = run_server(ps, arr)
        phase(f"serving: first {compare} requests one at a time, plain FP64")
        t0 = time.perf_counter()
        free_at, lat1, ok1 = 0.0, [], 0
        for a, p in zip(arr, ps):
            start = max(a, free_at)
            while time.perf_counter() - t0 < start:
                time.sleep(0.0002)
            r = ibb.minimize(p, fetch_boxes=False, incremental=False, max_sweeps=max_sweeps)
            ok1 += r.status == ibb.OK
            if len(lat1) % 16 == 15:
                phase(f"serving: one at a time, {len(lat1) + 1} of {compare} requests done")
            free_at = time.perf_counter() - t0
            lat1.append(free_at - a)
        lat1 = np.array(lat1)
        out["first_requests"] = {
            "requests": compare, "arrival_rate": round(lam, 2),
            "server": {"problems_per_s": round(compare / spanc, 2), "p50_ms": pct(latc, 50), "p99_ms": pct(latc, 99),
                       "converged": int(convc.sum())},
            "one_at_a_time_plain_fp64": {"problems_per_s": round(compare / (free_at - arr[0]), 2),
                                         "p50_ms": pct(lat1, 50), "p99_ms": pct(lat1, 99), "converged": int(ok1)}}
    return out


if __name__ == "__main__":
    sys.exit(main())
