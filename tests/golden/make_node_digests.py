"""Write the stored node-value digests under tests/golden/nodes_*.json from the oracle alone.

Usage:  python tests/golden/make_node_digests.py [group ...] [--procs N]
        groups: deg20 curve40 arrangement serving capacity polar (default: all)

Full-size parity without a full-size Bareiss run.  For a case (f, g) with
R = res(f, g; y) (the operands are (f, f_y) for kind disc and (f_x, f_y) for
kind polar):
  * D - 1 = oracle.bounds.degree_bound(f, g) bounds deg R, so the D values
    R(0), ..., R(D-1) determine R (Section 2: R is a polynomial in x; the
    specialisation R(a) = det S(f(a, y), g(a, y)) keeps the formal degrees);
  * modulo a prime q those values are det S(a) mod q, which the oracle computes
    one node at a time (oracle.resultant.resultant_at_mod: Gaussian elimination
    over F_q of the specialised Sylvester matrix);
  * primes q_1..q_K (the largest primes below 2^255, descending) are taken
    until their product Q exceeds 2^8 * B with B = oracle.bounds.coeff_bound,
    which bounds every coefficient of R.
A result R' with deg R' <= D - 1, max |coef R'| < Q / 2 and R'(a) = R(a)
mod q_k for every node a and every k equals R coefficient for coefficient
(Chinese remaindering of the interpolants, then the symmetric range).

Only digests are stored: for each q_k, sha256 of the decimal node values
"v_0,v_1,...,v_{D-1}" (v_a in [0, q_k)), plus a few plain values for
diagnostics.  Inputs are rebuilt from paper_1201_1548_amd.synth (which holds no
resultant arithmetic) and their digest is stored beside the values.  Nothing
here calls the library.
"""

import hashlib
import json
import math
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.bounds import coeff_bound, degree_bound  # noqa: E402
from oracle.resultant import bi_diff_y, bi_tdeg, bi_trim, resultant_at_mod  # noqa: E402
from oracle.subresultants import bi_diff_x  # noqa: E402
from paper_1201_1548_amd import synth  # noqa: E402
from tests.golden.make_golden import input_digest  # noqa: E402

PRIME_BITS = 255
MARGIN_BITS = 8
DEG20_PAIRS = [1, 2, 37, 64, 100, 128, 200, 255]
CAPACITY_MN = [(23, 9), (9, 23), (24, 4), (31, 31), (31, 2), (32, 6), (5, 0), (0, 7), (1, 1)]
GROUPS = ("deg20", "curve40", "arrangement", "serving", "capacity", "polar")


# ----------------------------------------------------------------------------
# case specifications -> inputs (shared with the tests)

def build_inputs(spec):
    """(kind, F, G) for a case spec; G is f_y for a discriminant and a polar
    resultant (whose first Sylvester operand is f_x: see ``operands``)."""
    gen = spec["gen"]
    args = spec.get("args", [])
    kw = spec.get("kw", {})
    if gen == "arrangement_pair":
        curves, pairs = _arrangement()
        i, j = pairs[args[0]]
        F, G = curves[i], curves[j]
    elif gen == "arrangement_curve":
        F, G = _arrangement()[0][args[0]], None
    elif gen == "poisson_request":
        req = _poisson()[args[0]]
        F, G = req["f"], req["g"]
    else:
        out = getattr(synth, gen)(*args, **kw)
        F, G = out if isinstance(out, tuple) else (out, None)
    kind = spec["kind"]
    if kind in ("disc", "polar"):
        return kind, F, bi_diff_y(F)
    return kind, F, G


def operands(kind, F, G):
    """The two Sylvester operands of a case from ``build_inputs``'s output."""
    return (bi_diff_x(F), G) if kind == "polar" else (F, G)


_CACHE = {}


def _arrangement():
    if "arr" not in _CACHE:
        _CACHE["arr"] = synth.arrangement_batch(0)
    return _CACHE["arr"]


def _poisson():
    if "poi" not in _CACHE:
        _CACHE["poi"] = synth.poisson_requests(0, n=2000)
    return _CACHE["poi"]


def node_digest(values):
    return hashlib.sha256(",".join(str(int(v)) for v in values).encode()).hexdigest()


def primes_below(bits, count):
    """The `count` largest primes below 2^bits, descending."""
    import sympy
    out = []
    q = 1 << bits
    while len(out) < count:
        q = sympy.prevprime(q)
        out.append(q)
    return out


def primes_for(bound):
    """Fewest of the descending primes below 2^PRIME_BITS whose product exceeds 2^MARGIN_BITS * bound."""
    need = max(bound, 1).bit_length() + MARGIN_BITS
    k = max(1, math.ceil(need / (PRIME_BITS - 1)))
    while True:
        ps = primes_below(PRIME_BITS, k)
        if math.prod(ps) > (bound << MARGIN_BITS):
            return ps
        k += 1


def load_group(group):
    with open(os.path.join(HERE, "nodes_%s.json" % group)) as fh:
        return json.load(fh)


# ----------------------------------------------------------------------------
# case selection

def cases_for(group):
    if group == "deg20":
        return [{"name": "deg20_pair_%d" % i, "gen": "pair_deg20", "args": [i], "kind": "res"} for i in DEG20_PAIRS]
    if group == "curve40":
        return [
            {"name": "curve_deg40_dense", "gen": "curve_deg40", "args": [0], "kind": "disc"},
            {"name": "curve_deg40_g2_hk", "gen": "singular_curve_deg40", "args": [0], "kind": "disc"},
            {"name": "curve_deg40_g2_hk2", "gen": "singular_curve_deg40", "args": [0],
             "kw": {"square_k": True, "dk": 10}, "kind": "disc"},
        ]
    if group == "capacity":
        return [{"name": "capacity_%d_%d" % (m, n), "gen": "random_rect", "args": [900 + 37 * m + n, m, 2, n, 1, 20],
                 "kind": "res"} for m, n in CAPACITY_MN]
    if group == "arrangement":
        return _arrangement_cases()
    if group == "serving":
        return _serving_cases()
    if group == "polar":
        curves, _ = _arrangement()
        big = max(range(len(curves)), key=lambda i: (bi_tdeg(curves[i]), _bits(curves[i])))
        return [
            {"name": "polar_curve_deg40_dense", "gen": "curve_deg40", "args": [0], "kind": "polar"},
            {"name": "polar_curve_deg40_g2_hk2", "gen": "singular_curve_deg40", "args": [0],
             "kw": {"square_k": True, "dk": 10}, "kind": "polar"},
            {"name": "polar_arrangement_curve_%d" % big, "gen": "arrangement_curve", "args": [big], "kind": "polar",
             "note": "total degree %d, %d-bit coefficients" % (bi_tdeg(curves[big]), _bits(curves[big]))},
            {"name": "polar_curve_deg12", "gen": "curve_deg40", "args": [5], "kw": {"tdeg": 12, "bits": 16},
             "kind": "polar"},
        ]
    raise ValueError(group)


def _bits(F):
    return max((abs(c).bit_length() for r in F for c in r), default=0)


def _arrangement_cases():
    """Eight of the 3800 pairs: the one with the largest coefficient bound
    (the largest prime count of the batch), the smallest, and six spread over
    the range of total degrees and coefficient sizes."""
    curves, pairs = _arrangement()
    td = [bi_tdeg(c) for c in curves]
    bt = [_bits(c) for c in curves]
    proxy = [((td[i] + td[j]) * (bt[i] + bt[j]), k) for k, (i, j) in enumerate(pairs)]
    proxy.sort()
    top = [k for _, k in proxy[-200:]]
    largest = max(top, key=lambda k: coeff_bound(curves[pairs[k][0]], curves[pairs[k][1]]))
    n = len(proxy)
    picks = [proxy[0][1]] + [proxy[int(n * f)][1] for f in (0.1, 0.3, 0.5, 0.7, 0.85, 0.95)] + [largest]
    out = []
    for k in picks:
        i, j = pairs[k]
        out.append({"name": "arrangement_pair_%d" % k, "gen": "arrangement_pair", "args": [k], "kind": "res",
                    "note": "curves %d, %d: total degrees %d, %d; coefficient bits %d, %d" % (
                        i, j, td[i], td[j], bt[i], bt[j])})
    return out


def _serving_cases():
    """Four of the first 300 serving requests (two resultants, two
    discriminants) whose coefficient bound exceeds 2^4300, so that more than
    128 word primes are needed; the cheapest for the oracle among those."""
    reqs = _poisson()[:300]
    cand = []
    for k, req in enumerate(reqs):
        spec = {"gen": "poisson_request", "args": [k], "kind": req["kind"]}
        _, F, G = build_inputs(spec)
        B = coeff_bound(F, G)
        if B.bit_length() < 4300:
            continue
        D = degree_bound(F, G) + 1
        r = len(bi_trim(F)) + len(bi_trim(G)) - 2
        cost = D * (B.bit_length() // 250 + 1) * r ** 3
        cand.append((cost, k, req["kind"], req["tdeg"], req["bits"]))
    cand.sort()
    out = []
    for kind in ("res", "disc"):
        for cost, k, kd, tdeg, bits in [c for c in cand if c[2] == kind][:2]:
            out.append({"name": "serving_request_%d" % k, "gen": "poisson_request", "args": [k], "kind": kd,
                        "note": "total degree %d, %d-bit coefficients" % (tdeg, bits)})
    return out


# ----------------------------------------------------------------------------
# the oracle runs

def _task(spec, q, a0, a1):
    A, B = operands(*build_inputs(spec))
    return [resultant_at_mod(A, B, a, q) for a in range(a0, a1)]


def run_group(group, procs):
    cases = cases_for(group)
    plans = []
    tasks = []
    for spec in cases:
        kind, F, G = build_inputs(spec)
        D = degree_bound(*operands(kind, F, G)) + 1
        B = coeff_bound(*operands(kind, F, G))
        ps = primes_for(B)
        plans.append((spec, F, G, D, B, ps))
        chunk = max(1, D // 8)
        for qi, q in enumerate(ps):
            for a0 in range(0, D, chunk):
                tasks.append((spec, q, a0, min(D, a0 + chunk)))
        print("%s: D = %d, bound 2^%d, %d primes" % (spec["name"], D, B.bit_length(), len(ps)), flush=True)
    t0 = time.time()
    ctx = mp.get_context("fork")
    with ctx.Pool(procs) as pool:
        chunks = pool.starmap(_task, tasks, chunksize=1)
    dt = time.time() - t0
    results = {}
    for (spec, q, a0, a1), vals in zip(tasks, chunks):
        results.setdefault((spec["name"], q), {})[a0] = vals
    out = []
    for spec, F, G, D, B, ps in plans:
        digests, samples = [], []
        for qi, q in enumerate(ps):
            parts = results[(spec["name"], q)]
            vals = [v for a0 in sorted(parts) for v in parts[a0]]
            assert len(vals) == D
            digests.append(node_digest(vals))
            if qi == 0:
                samples = [[a, str(vals[a])] for a in sorted({0, 1, D // 2, D - 1})]
        rec = dict(spec)
        rec.update({
            "inputs_sha256": input_digest(F, G if spec["kind"] == "res" else None),
            "D": D,
            "coeff_bound_bits": B.bit_length(),
            "primes": [str(q) for q in ps],
            "digests": digests,
            "samples_prime0": samples,
        })
        out.append(rec)
    doc = {
        "about": "Digests of R(a) mod q for a = 0..D-1 (R = res(f, g; y), res(f, f_y; y) for kind disc, "
                 "res(f_x, f_y; y) for kind polar), "
                 "written by tests/golden/make_node_digests.py with oracle.resultant.resultant_at_mod, "
                 "oracle.bounds.degree_bound and oracle.bounds.coeff_bound only.",
        "group": group,
        "oracle_seconds": round(dt, 1),
        "processes": procs,
        "cases": out,
    }
    path = os.path.join(HERE, "nodes_%s.json" % group)
    with open(path, "w") as fh:
        json.dump(doc, fh, indent=1)
    print("wrote %s (%d cases, %.0f s with %d processes)" % (path, len(out), dt, procs), flush=True)


def main(argv):
    procs = max(1, (os.cpu_count() or 2) - 1)
    groups = []
    it = iter(argv)
    for a in it:
        if a == "--procs":
            procs = int(next(it))
        else:
            groups.append(a)
    for g in groups or GROUPS:
        run_group(g, procs)


if __name__ == "__main__":
    main(sys.argv[1:])
