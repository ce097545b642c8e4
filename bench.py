#!/usr/bin/env python3
"""Benchmark: exact bivariate resultants per second on one MI355X.

Workload: N independent pairs (default 256) of dense total-degree-20 bivariate
polynomials with uniform 32-bit signed coefficients (seeds 2000..2000+N-1),
res(f, g; y) in Z[x] of every pair.  One step = one batched call over all N
pairs with inputs and outputs resident in HBM (every stage of the path:
reduction, evaluation + univariate resultants, interpolation, mixed-radix
conversion, limb assembly).  The plain path (one library call per pair) is
timed on the same pairs and checked bit-exact against the batched results.

Prints one JSON line (see the fields at the end of main()).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bivariate resultants/sec (deg-20, 32-bit) batched vs plain; INT32 VALU % peak; p99"

# Full-rate 32-bit VALU peak: 64 lanes per clock per CU (a wave64 instruction
# issues in 4 cycles on a 16-lane SIMD, 4 SIMDs per CU; the library's issue
# probe measures 4.6 cycles for v_mul_lo_u32 and v_mad_u64_u32, so the
# multiplies run at this rate; only adds reach twice it), 256 CUs, 2.4 GHz.
LANES_PER_CU_CLOCK = 64


def int_peak_tops(dev):
    return dev["cus"] * LANES_PER_CU_CLOCK * dev["clock_khz"] * 1e3 / 1e12


TRAFFIC_SOURCES = ("kernels.hip", "kernels.hpp", "job.hpp", "modp.hpp")


def kernel_source_digest():
    """sha256 over the device sources of the library (fixed order)."""
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1201_1548_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_counters(kind, kernel, workload, field):
    """A figure of the committed rocprofv3 counter summary
    profiles/<kind>_<kernel>_<workload>.md (a line 'field: value'), or None when
    the summary is missing or was taken on other kernel sources (its
    source_sha256 line differs from the current device sources)."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s.md" % (kind, kernel, workload))
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith(("source_sha256", field)):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_sha256") != kernel_source_digest() or field not in fields:
        return None
    return float(fields[field])


def stored_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` (profiles/traffic_*.md)."""
    v = stored_counters("traffic", kernel, workload, "hbm_bytes_per_launch")
    return None if v is None else int(v)


def model_mulmods(rowdeg_f, rowdeg_g):
    """Modular products of one (prime, point) instance in the method's own
    terms: one product per coefficient for the evaluation of f(a, y) and
    g(a, y), and two per Sylvester-entry elimination for the 2 m n entries of a
    normal remainder sequence (a reference count, not the kernel's
    instructions)."""
    T = sum(d + 1 for d in rowdeg_f if d >= 0) + sum(d + 1 for d in rowdeg_g if d >= 0)
    m, n = len(rowdeg_f) - 1, len(rowdeg_g) - 1
    return T + 2 * m * n


def cpu_baseline(pairs, D, budget_s=15.0):
    """The oracle on a bounded sample: R(a) = det S(f(a,y), g(a,y)) (integer
    Bareiss) at as many points of the first pairs as fit the budget, on a
    process pool over the host cores.  A full resultant needs D such points
    (interpolation is not counted, which favours the CPU)."""
    import multiprocessing as mp
    from oracle.resultant import resultant_at

    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(16, affinity))
    F, G = pairs[0]
    t0 = time.time()
    resultant_at(F, G, 0)
    per_point = max(time.time() - t0, 1e-4)
    npts = max(cores, int(budget_s * cores / per_point))
    npts = min(npts, 64 * cores)
    tasks = [(pairs[(i // D) % len(pairs)], i % D) for i in range(npts)]
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        t0 = time.time()
        pool.starmap(_point, tasks, chunksize=max(1, npts // (4 * cores)))
        dt = time.time() - t0
    return {
        "value": npts / dt / D,
        "unit": "resultants/s",
        "cores": cores,
        "host_cpu_count": os.cpu_count(),
        "host_cpus_allowed": affinity,
        "kind": "oracle",
        "sample": "%d evaluation points R(a) of the dense total-degree-20 pairs by the oracle's integer Bareiss "
                  "determinant of the specialised Sylvester matrix, %d processes; value = points/s / %d "
                  "points per resultant (interpolation not counted)" % (npts, cores, D),
    }


def _point(pair, a):
    from oracle.resultant import resultant_at
    F, G = pair
    return resultant_at(F, G, a)


def _percentile(v, q):
    v = sorted(v)
    if not v:
        return None
    i = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[i]


def bench_arrangement(args):
    """Arrangement: 400 curves (total degree U{4..30}, bits U{8..64}), all pairs in
    seeded groups of 20 (3800 resultants); one batched call vs one call per pair."""
    import torch
    import paper_1201_1548_amd as br
    from paper_1201_1548_amd import synth

    curves, pairs = synth.arrangement_batch(0)
    jobs = [("res", curves[i], curves[j], "y") for i, j in pairs]
    torch.cuda.set_device(0)
    batch = br.DeviceBatch(jobs)
    br.set_schedule(args.schedule)
    chosen = batch.autotune(reps=1) if args.schedule == "auto" else args.schedule
    batch.run()
    torch.cuda.synchronize()
    res = batch.results()
    for _ in range(args.warmup):
        batch.run()
    torch.cuda.synchronize()
    br.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, launches = br.kernel_time()
    br.set_timing(False)
    batch.run_each()
    torch.cuda.synchronize()
    exact_plain = batch.results() == res
    t0 = time.perf_counter()
    batch.run_each()
    torch.cuda.synchronize()
    dtp = time.perf_counter() - t0
    n = len(jobs)
    return {
        "metric": "arrangement pair resultants/sec, batched vs plain",
        "value": round(n * args.steps / dt, 2), "unit": "resultants/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "arrangement: 400 dense curves, total degree U{4..30}, coefficient bits U{8..64}, "
                               "all pairs within 20 seeded groups of 20 (3800 res_y)", "pairs": n},
        "plain": {"value": round(n / dtp, 2), "unit": "resultants/s", "ms_per_pair": round(dtp / n * 1e3, 3)},
        "batched_over_plain": round((n * args.steps / dt) / (n / dtp), 2),
        "schedule": chosen,
        "timed_kernels_ms_per_step": round(kms / max(launches, 1), 3),
        "bit_exact": {"batched_vs_plain": exact_plain},
    }


def bench_serving(args):
    """Serving: Poisson stream of resultant/discriminant requests (total degree
    log-uniform in [5, 64], bits U{10..128}); the continuous-batching server vs
    a plain server that runs one library call per request in arrival order."""
    import threading
    import paper_1201_1548_amd as br
    from paper_1201_1548_amd import synth

    nreq = args.requests
    probe = synth.poisson_requests(0, n=min(40, nreq), qps=1.0)

    def plain_call(r):
        return br.discriminant(r["f"]) if r["kind"] == "disc" else br.resultant(r["f"], r["g"])

    plain_call(probe[0])
    t0 = time.perf_counter()
    for r in probe:
        plain_call(r)
    service = (time.perf_counter() - t0) / len(probe)
    qps = args.qps or 0.7 / service
    reqs = synth.poisson_requests(0, n=nreq, qps=qps)

    def run_plain():
        out, lat = [None] * nreq, [0.0] * nreq
        start = time.perf_counter()
        for i, r in enumerate(reqs):
            now = time.perf_counter() - start
            if now < r["t"]:
                time.sleep(r["t"] - now)
            out[i] = plain_call(r)
            lat[i] = time.perf_counter() - start - r["t"]
        return out, lat, time.perf_counter() - start

    def run_server():
        out, lat = [None] * nreq, [0.0] * nreq
        with br.Server(hbm_budget_bytes=args.budget_gib << 30, max_slots=args.slots) as srv:
            tickets = [None] * nreq
            ready = threading.Semaphore(0)
            start = time.perf_counter()

            def submitter():
                for i, r in enumerate(reqs):
                    now = time.perf_counter() - start
                    if now < r["t"]:
                        time.sleep(r["t"] - now)
                    tickets[i] = srv.submit(r["kind"], r["f"], r["g"])
                    ready.release()

            th = threading.Thread(target=submitter)
            th.start()
            for i in range(nreq):
                ready.acquire()
                out[i], lat[i] = srv.wait(tickets[i])
            th.join()
            total = time.perf_counter() - start
        return out, lat, total

    out_s, lat_s, tot_s = run_server()
    out_p, lat_p, tot_p = run_plain()
    return {
        "metric": "serving: resultant/discriminant requests/sec with p50/p99 latency",
        "value": round(nreq / tot_s, 2), "unit": "requests/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(tot_s * 1e3, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "serving: Poisson arrivals, total degree round(exp(U[ln5, ln64])), "
                               "coefficient bits U{10..128}, resultant or discriminant 50/50",
                   "requests": nreq, "qps": round(qps, 2), "hbm_budget_gib": args.budget_gib,
                   "slots": args.slots},
        "p50_ms": round(_percentile(lat_s, 50) * 1e3, 2), "p99_ms": round(_percentile(lat_s, 99) * 1e3, 2),
        "plain": {"value": round(nreq / tot_p, 2), "unit": "requests/s",
                  "p50_ms": round(_percentile(lat_p, 50) * 1e3, 2),
                  "p99_ms": round(_percentile(lat_p, 99) * 1e3, 2),
                  "mean_service_ms": round(service * 1e3, 2)},
        "bit_exact": {"server_vs_plain": out_s == out_p},
    }


def read_golden(path):
    """Coefficients stored in a golden file (text: '#' comments, 'inputs' and
    'degree' lines, then one decimal coefficient per line)."""
    coeffs = []
    with open(path) as fh:
        for line in fh:
            if line.startswith(("#", "inputs ", "degree ")) or not line.strip():
                continue
            coeffs.append(int(line))
    return coeffs


def _zx_derivative(a):
    d = [i * a[i] for i in range(1, len(a))]
    while d and d[-1] == 0:
        d.pop()
    return d


def _zx_mul(a, b):
    """Product in Z[x] by Kronecker substitution (signed digits)."""
    if not a or not b:
        return []
    k = max(abs(c) for c in a).bit_length() + max(abs(c) for c in b).bit_length() + min(len(a), len(b)).bit_length() + 2
    v = sum(c << (k * i) for i, c in enumerate(a)) * sum(c << (k * i) for i, c in enumerate(b))
    out = []
    for _ in range(len(a) + len(b) - 1):
        c = v & ((1 << k) - 1)
        if c >> (k - 1):
            c -= 1 << k
        out.append(c)
        v = (v - c) >> k
    while out and out[-1] == 0:
        out.pop()
    return out


def bench_autotune(args):
    """The schedule space per workload shape: every schedule (staged, fused,
    Schur) timed on the same device batch, checked bit-exact against the staged
    results, and the autotuner's choice (bires_autotune, the best of three
    timed rounds per schedule) next to the fastest measured one."""
    import torch
    import paper_1201_1548_amd as br
    from paper_1201_1548_amd import synth

    torch.cuda.set_device(0)
    shapes = {}
    shapes["deg20_batch256"] = [("res",) + synth.pair_deg20(s) + ("y",) for s in range(256)]
    shapes["curve40_disc3"] = [("disc", synth.curve_deg40(0), None, "y"),
                               ("disc", synth.singular_curve_deg40(0), None, "y"),
                               ("disc", synth.singular_curve_deg40(0, square_k=True, dk=10), None, "y")]
    curves, pairs = synth.arrangement_batch(0)
    shapes["arrangement_3800"] = [("res", curves[i], curves[j], "y") for i, j in pairs]
    reqs = synth.poisson_requests(0, n=64, qps=1.0)
    shapes["serving_batch64"] = [(r["kind"], r["f"], r["g"], "y") for r in reqs]
    cases = {}
    agree = 0
    for name, jobs in shapes.items():
        batch = br.DeviceBatch(jobs)
        br.set_schedule("staged")
        batch.run()
        torch.cuda.synchronize()
        ref = batch.results()
        times = {}
        for sched in ("staged", "fused", "schur"):
            br.set_schedule(sched)
            batch.run()
            torch.cuda.synchronize()
            ok = batch.results() == ref
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                batch.run()
            torch.cuda.synchronize()
            times[sched] = {"ms_per_step": round((time.perf_counter() - t0) / reps * 1e3, 3), "bit_exact": ok}
        br.set_schedule("auto")
        chosen = batch.autotune(reps=3)
        fastest = min(times, key=lambda k: times[k]["ms_per_step"])
        agree += chosen == fastest
        cases[name] = {"jobs": len(jobs), "schedules": times, "autotuner": chosen, "fastest": fastest}
    br.set_schedule(args.schedule)
    return {
        "metric": "schedule space per workload shape: step time of each schedule and the autotuner's choice",
        "value": agree, "unit": "shapes where the autotuner chose the fastest schedule", "n_gpus": 1,
        "steps": 3, "warmup": 1, "ms_per_step": cases["deg20_batch256"]["schedules"][cases["deg20_batch256"]["autotuner"]]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "the deg-20 bench batch, the three degree-40 discriminants, the 3800 arrangement "
                               "pairs and a batch of the first 64 serving requests"},
        "cases": cases,
    }


def bench_curve40(args):
    """Curve analysis: res(f, f_y; y) of a dense total-degree-40 curve (16-bit
    coefficients), gcd(R, R') and the square-free decomposition of R; per-call
    wall time."""
    import torch
    import paper_1201_1548_amd as br
    from paper_1201_1548_amd import synth

    torch.cuda.set_device(0)
    out = {}
    for name, F in (("dense", synth.curve_deg40(0)),
                    ("g2_hk", synth.singular_curve_deg40(0)),
                    ("g2_hk2", synth.singular_curve_deg40(0, square_k=True, dk=10))):
        br.discriminant(F)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            R = br.discriminant(F)
        td = (time.perf_counter() - t0) / args.steps
        dR = _zx_derivative(R)
        h = br.gcd(R, dR)  # warm-up: tables for this prime set
        t0 = time.perf_counter()
        for _ in range(args.steps):
            h = br.gcd(R, dR)
        tg = (time.perf_counter() - t0) / args.steps
        u, fs = br.squarefree(R)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            u, fs = br.squarefree(R)
        tq = (time.perf_counter() - t0) / args.steps
        # the same discriminant through the Schur schedule (wavefront per
        # instance), bit-exact against the staged result
        br.set_schedule("schur")
        try:
            Rs_ = br.discriminant(F)
            t0 = time.perf_counter()
            for _ in range(args.steps):
                Rs_ = br.discriminant(F)
            tds = (time.perf_counter() - t0) / args.steps
        finally:
            br.set_schedule("auto")
        # Q = res(f_x, f_y; y), the psc's of (f, f_y) modulo one prime, and the
        # N^- / N^+ test with R* = prod a_i
        Q = br.polar_resultant(F)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Q = br.polar_resultant(F)
        tQ = (time.perf_counter() - t0) / args.steps
        p0, rows = br.psc(F, kind="disc")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            p0, rows = br.psc(F, kind="disc")
        tP = (time.perf_counter() - t0) / args.steps
        Rstar = [1]
        for a in fs:
            Rstar = _zx_mul(Rstar, a)
        nb = br.fiber_bounds(F, Rstar, len(R) - 1)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            nb = br.fiber_bounds(F, Rstar, len(R) - 1)
        tN = (time.perf_counter() - t0) / args.steps
        # R = u * prod a_i^i, checked exactly
        prod = [u]
        for i, a in enumerate(fs):
            for _ in range(i + 1):
                prod = _zx_mul(prod, a)
        out[name] = {"disc_ms": round(td * 1e3, 2), "deg_R": len(R) - 1, "gcd_ms": round(tg * 1e3, 2),
                     "deg_gcd": len(h) - 1, "squarefree_ms": round(tq * 1e3, 2),
                     "squarefree_degrees": [len(a) - 1 for a in fs], "squarefree_exact": prod == R,
                     "disc_schur_ms": round(tds * 1e3, 2), "disc_schur_exact": Rs_ == R,
                     "polar_Q_ms": round(tQ * 1e3, 2), "deg_Q": len(Q) - 1,
                     "psc_mod_p_ms": round(tP * 1e3, 2), "psc_count": len(rows), "psc_prime": p0,
                     "fiber_bounds_ms": round(tN * 1e3, 2), "n_minus": nb[0], "n_plus": nb[1],
                     "fiber_flags": nb[2]}
    return {
        "metric": "curve-analysis resultant res(f, f_y; y), gcd(R, R'), square-free decomposition, Q = res(f_x, f_y; y), "
                  "psc's mod p and the N^-/N^+ test: wall time (degree-40 curves)",
        "value": round(1e3 / out["dense"]["disc_ms"], 2), "unit": "discriminants/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": out["dense"]["disc_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "curve analysis: dense total degree 40, 16-bit coefficients; g^2 + h k with dense "
                               "degree-20 factors, 8-bit; g^2 + h k^2 (k degree 10)"},
        "cases": out,
    }


def bench_rates(args):
    """VALU issue cost per wave64 instruction (the library's probe kernels),
    the figures behind the roofline's instruction model."""
    import torch
    import paper_1201_1548_amd as br
    torch.cuda.set_device(0)
    r = br.issue_rates()
    return {"metric": "VALU issue cycles per wave64 instruction per SIMD", "value": r["v_mad_u64_u32"],
            "unit": "cycles (v_mad_u64_u32)", "rates": {k: round(v, 3) for k, v in r.items()},
            "device": br.device_info()}


def bench_copy(args):
    """Calibration for the HBM counters: a plain device copy of a known size
    (torch's copy kernel), repeated `steps` times."""
    import torch
    n = 1 << 28  # 1 GiB of int32
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"metric": "device copy bandwidth (counter calibration)", "value": round(2 * 4 * n * args.steps / dt / 1e9, 1),
            "unit": "GB/s", "bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n, "copies": args.steps + 1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--pairs", type=int, default=256)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain path (profiling runs)")
    ap.add_argument("--no-graphs", action="store_true", help="skip the graph-replay leg")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the leg with two batches in flight (the headline is then the synchronous leg)")
    ap.add_argument("--eval-kernel", default="auto", choices=["auto", "lds"],
                    help="evaluation + elimination kernel of the staged schedule")
    ap.add_argument("--workload", default="deg20",
                    choices=["deg20", "curve40", "arrangement", "serving", "autotune", "copy", "rates"])
    ap.add_argument("--schedule", default="auto", choices=["auto", "staged", "fused"])
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--qps", type=float, default=0.0)
    ap.add_argument("--budget-gib", type=int, default=32)
    ap.add_argument("--slots", type=int, default=64)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (each job runs on one "
              "device; a batch would shard by jobs, a large job by primes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.workload != "deg20":
        fn = {"curve40": bench_curve40, "arrangement": bench_arrangement, "serving": bench_serving,
              "autotune": bench_autotune, "copy": bench_copy, "rates": bench_rates}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return

    import paper_1201_1548_amd as br
    from paper_1201_1548_amd import synth

    n = args.pairs
    pairs = [synth.pair_deg20(s) for s in range(n)]
    D, P, _ = br.plan(pairs[0][0], pairs[0][1])
    # the CPU leg runs first, in forked workers, before anything touches the GPU
    cpu = None if args.no_cpu else cpu_baseline(pairs, D)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    dev = br.device_info()
    batch = br.DeviceBatch([("res", F, G, "y") for F, G in pairs])
    br.set_eval_kernel(args.eval_kernel)
    br.set_schedule(args.schedule)
    chosen = batch.autotune(reps=2) if args.schedule == "auto" else args.schedule

    # correctness gate: batched == plain == stored oracle values
    batch.run()
    torch.cuda.synchronize()
    res_batch = batch.results()
    golden = os.path.join(ROOT, "tests", "golden", "deg20_res_0.txt")
    exact_golden = None
    if os.path.exists(golden):
        exact_golden = read_golden(golden) == res_batch[0]

    for _ in range(args.warmup):
        batch.run()
    torch.cuda.synchronize()
    br.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, launches = br.kernel_time()
    host_us, host_calls = br.host_time()
    br.set_timing(False)
    sync_value = n * args.steps / dt
    sync_ms = dt / args.steps * 1e3

    # the same steps with two batches in flight (bires_resultant_batch_async):
    # step k+1's row scan and planning overlap step k's kernels.  Two device
    # batches of the same jobs alternate, so calls in flight never share
    # output buffers.
    pipe = None
    if not args.no_pipeline:
        twin = br.DeviceBatch([("res", F, G, "y") for F, G in pairs])
        bs = (batch, twin)
        for k in range(max(args.warmup, 2)):
            bs[k % 2].run_async()
            bs[k % 2].wait()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prev = None
        for k in range(args.steps):
            b = bs[k % 2]
            b.run_async()
            if prev is not None:
                prev.wait()
            prev = b
        prev.wait()
        torch.cuda.synchronize()
        dtp_ = time.perf_counter() - t0
        pipe_exact = batch.results() == res_batch and twin.results() == res_batch
        pipe = {"value": round(n * args.steps / dtp_, 2), "ms_per_step": round(dtp_ / args.steps * 1e3, 3),
                "bit_exact": pipe_exact}
        del twin, bs
    # headline: the steps with two batches in flight when they are bit-exact
    # (every step is still one whole pass over one batch), else one at a time
    if pipe is not None and pipe["bit_exact"]:
        value, dt = n * args.steps / dtp_, dtp_
    else:
        value = sync_value

    # the same steps replayed from a captured HIP graph (checked bit-exact)
    graph = None
    if not args.no_graphs:
        br.set_graphs(True)
        try:
            batch.run()
            torch.cuda.synchronize()
            graph_exact = batch.results() == res_batch
            t0 = time.perf_counter()
            for _ in range(args.steps):
                batch.run()
            torch.cuda.synchronize()
            dtg = time.perf_counter() - t0
            caps, reps = br.graph_stats()
        finally:
            br.set_graphs(False)
        graph = {"value": round(n * args.steps / dtg, 2), "ms_per_step": round(dtg / args.steps * 1e3, 3),
                 "bit_exact": graph_exact, "captures": caps, "replays": reps}

    # the batch under each schedule the autotuner chooses from (a few steps
    # each, checked bit-exact): why the tuned choice is the one it is
    schedules = {}
    for name in ("staged", "fused", "schur"):
        br.set_schedule(name)
        try:
            batch.run()
            torch.cuda.synchronize()
            ok = batch.results() == res_batch
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                batch.run()
            torch.cuda.synchronize()
            schedules[name] = {"ms_per_step": round((time.perf_counter() - t0) / reps * 1e3, 3), "bit_exact": ok}
        finally:
            br.set_schedule(args.schedule)

    # plain path: one call per pair, same pairs, same buffers
    exact_plain = None
    if not args.no_plain:
        batch.run_each()
        torch.cuda.synchronize()
        exact_plain = batch.results() == res_batch
    plain_value = dtp = None
    if args.plain_steps > 0 and not args.no_plain:
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            batch.run_each()
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        plain_value = n * args.plain_steps / dtp

    # roofline of the dominant kernel (evaluation + univariate resultants):
    # integer lane-ops per (prime, point) instance from the committed SQ
    # counters (integer VALU instructions per wave; one lane per instance),
    # times the instances of one launch, over the live launch time
    workload = "deg20_batch%d" % n
    instances = P * D * n
    avg_ms = kms / max(launches, 1)
    peak = int_peak_tops(dev)
    per_inst = stored_counters("valu", "k_eval_elim_rg24", workload, "int_lane_ops_per_instance")
    achieved = None if per_inst is None else per_inst * instances / (avg_ms / 1e3) / 1e12
    rowdeg = [20 - j for j in range(21)]
    mulmods = model_mulmods(rowdeg, rowdeg)
    roofline = {
        "bound": "alu",
        "achieved": None if achieved is None else round(achieved, 3),
        "peak": round(peak, 2),
        "unit": "T int32-lane-op/s",
        "frac": None if achieved is None else round(achieved / peak, 4),
        "traffic": stored_traffic("k_eval_elim_rg24", workload),
        "traffic_unit": "bytes per launch",
        "kernel": "k_eval_elim_rg24 (+ k_eval_elim_fb)",
        "kernel_ms": round(avg_ms, 4),
        "instances_per_launch": instances,
        "int_lane_ops_per_instance": per_inst,
        "counters": "profiles/valu_k_eval_elim_rg24_%s.md" % workload,
        "model_mulmods_per_instance": mulmods,
        "model_mulmod_rate_T_per_s": round(mulmods * instances / (avg_ms / 1e3) / 1e12, 3),
    }

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "resultants/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "batch of %d pairs of dense total-degree-20 polynomials in Z[x,y], "
                        "uniform 32-bit signed coefficients, res_y" % n,
            "pairs": n, "tdeg": 20, "coef_bits": 32, "points": D, "primes": P,
        },
        "plain": None if plain_value is None else {
            "value": round(plain_value, 2), "unit": "resultants/s",
            "ms_per_pair": round(dtp / (n * args.plain_steps) * 1e3, 3)},
        "batched_over_plain": None if plain_value is None else round(value / plain_value, 2),
        "schedule": chosen,
        "bit_exact": {"batched_vs_plain": exact_plain, "pair0_vs_oracle_golden": exact_golden},
        "device": dev,
        "headline_leg": "pipelined" if value != sync_value else "synchronous",
        "synchronous": {"value": round(sync_value, 2), "ms_per_step": round(sync_ms, 3)},
        "pipelined": pipe,
        "host_us_per_step": {k: round(v / max(host_calls, 1), 1) for k, v in host_us.items()},
        "graph_replay": graph,
        "schedules": schedules,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
