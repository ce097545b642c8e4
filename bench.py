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

# INT32 lane-op cost of the modular primitives in their minimal gfx950 form:
# Montgomery product = v_mad_u64_u32, v_mul_lo_u32, v_mad_u64_u32, v_sub, v_min;
# two-product dot (one reduction) = one more v_mad_u64_u32; add/sub mod p = 2.
OPS_MULMOD, OPS_DOT2, OPS_ADDMOD = 5, 6, 2
# 256 CUs x 128 32-bit lanes per clock (the vector width behind the
# 157.3 TFLOP/s fp32 figure: 2 flops x 128 x 256 x 2.4 GHz) x 2.4 GHz.
INT32_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12


def _pow_cost(e):
    return (e.bit_length() + bin(e).count("1")) if e > 0 else 0


def instance_ops(rowdeg_f, rowdeg_g):
    """Algorithmic INT32 lane-ops of one (prime, point) instance of the
    evaluation + univariate resultant kernel, for the generic case (no
    leading coefficient vanishes).  Counts the modular operations the method
    performs, not loop control or addressing."""
    mul = dot = add = 0
    for d in list(rowdeg_f) + list(rowdeg_g):     # Horner: multiply by a, add the coefficient
        mul += d + 1
        add += d + 1
    a, b = len(rowdeg_f) - 1, len(rowdeg_g) - 1
    if a < b:
        a, b = b, a
    while True:
        if b == 0:
            mul += _pow_cost(a) + 1
            break
        a0, kk = a, 0
        while a >= b:
            s = a - b
            mul += s
            dot += a - s
            a -= 1
            kk += 1
        e = a0 - a - kk * b
        mul += _pow_cost(abs(e)) + 1
        a, b = b, a
    mul += _pow_cost(2**31 - 3) + 2                 # one Fermat inverse, final product, output conversion
    return mul * OPS_MULMOD + dot * OPS_DOT2 + add * OPS_ADDMOD


def cpu_baseline(pairs, D, budget_s=15.0):
    """The oracle on a bounded sample: R(a) = det S(f(a,y), g(a,y)) (integer
    Bareiss) at as many points of the first pairs as fit the budget, on a
    process pool over the host cores.  A full resultant needs D such points
    (interpolation is not counted, which favours the CPU)."""
    import multiprocessing as mp
    from oracle.resultant import resultant_at

    cores = max(1, min(16, os.cpu_count() or 1))
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
        "kind": "oracle",
        "sample": "%d evaluation points R(a) of config-2 pairs by the oracle's integer Bareiss "
                  "determinant of the specialised Sylvester matrix, %d processes; value = points/s / %d "
                  "points per resultant (interpolation not counted)" % (npts, cores, D),
    }


def _point(pair, a):
    from oracle.resultant import resultant_at
    F, G = pair
    return resultant_at(F, G, a)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--pairs", type=int, default=256)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each job runs on one "
              "device; see the sharding notes in DESIGN.md). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import paper_1201_1548_amd as br
    from paper_1201_1548_amd import synth

    n = args.pairs
    pairs = [synth.config2_pair(s) for s in range(n)]
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

    # correctness gate: batched == plain == stored oracle values
    batch.run()
    torch.cuda.synchronize()
    res_batch = batch.results()
    golden = os.path.join(ROOT, "tests", "golden", "config2_res_0.txt")
    exact_golden = None
    if os.path.exists(golden):
        from tests.golden.make_golden import load
        exact_golden = load("config2_res_0.txt")[1] == res_batch[0]

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
    value = n * args.steps / dt

    # plain path: one call per pair, same pairs, same buffers
    batch.run_each()
    torch.cuda.synchronize()
    exact_plain = batch.results() == res_batch
    t0 = time.perf_counter()
    for _ in range(args.plain_steps):
        batch.run_each()
    torch.cuda.synchronize()
    dtp = time.perf_counter() - t0
    plain_value = n * args.plain_steps / dtp

    # roofline of the dominant kernel (evaluation + univariate resultants)
    rowdeg = [20 - j for j in range(21)]
    ops_per_instance = instance_ops(rowdeg, rowdeg)
    ops_launch = ops_per_instance * P * D * n
    avg_ms = kms / max(launches, 1)
    achieved = ops_launch / (avg_ms / 1e3) / 1e12
    roofline = {
        "bound": "alu",
        "achieved": round(achieved, 3),
        "peak": round(INT32_PEAK_TOPS, 1),
        "unit": "T int32-op/s",
        "frac": round(achieved / INT32_PEAK_TOPS, 4),
        "traffic": None,
        "kernel": "k_eval_elim",
        "kernel_ms": round(avg_ms, 4),
        "ops_per_launch": ops_launch,
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
            "workload": "config 2 batched: %d pairs of dense total-degree-20 polynomials in Z[x,y], "
                        "uniform 32-bit signed coefficients, res_y" % n,
            "pairs": n, "tdeg": 20, "coef_bits": 32, "points": D, "primes": P,
        },
        "plain": {"value": round(plain_value, 2), "unit": "resultants/s",
                  "ms_per_pair": round(dtp / (n * args.plain_steps) * 1e3, 3)},
        "batched_over_plain": round(value / plain_value, 2),
        "bit_exact": {"batched_vs_plain": exact_plain, "pair0_vs_oracle_golden": exact_golden},
        "device": dev,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
