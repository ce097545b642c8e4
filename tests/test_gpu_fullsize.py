"""Full-size bit-exact parity with the oracle on every workload shape, through
the launch configurations the benchmark times.

Each result is compared with the oracle's R(a) mod q at every node a = 0..D-1
for primes whose product exceeds twice the coefficient bound (tests/nodecheck.py),
which fixes R over Z; the oracle's values were stored as digests by
tests/golden/make_node_digests.py.  Covered:

* 8 of the 256 dense total-degree-20 pairs of the benchmark batch (device
  memory, plan reuse, the staged schedule), besides pair 0's stored full value;
  the persistent fused schedule's results of the whole batch equal them;
* the degree-40 curve-analysis resultants res(f, f_y; y) (D = 1561): the dense
  curve, g^2 + h k and g^2 + h k^2, with gcd(R, R') checked by its defining
  properties including its content;
* 8 pairs of the 3800-pair arrangement batch (total degrees 4..30, 8..64-bit
  coefficients, the pair with the largest prime count among them), from the
  whole batch under the staged and the fused schedule and as single calls;
* 4 serving requests that need more than 128 primes (the Garner route of the
  reconstruction) through the server, in a mix with other requests, and as
  single calls;
* the evaluation kernels' capacity boundaries (register array 24/32, LDS
  kernel, a zero y-degree), batched with each kernel, under the fused
  schedule and single.
The P > 128 route is also checked against the oracle's full Bareiss value on
low-y-degree pairs with 360..700-bit coefficients, alone and in mixed batches.
"""

import pytest

import paper_1201_1548_amd as br
from oracle import zx
from oracle.gcd import gcd_mod_p
from oracle.resultant import bi_diff_y, resultant_y
from paper_1201_1548_amd import synth
from tests import nodecheck
from tests.golden.make_golden import load
from tests.golden.make_node_digests import CAPACITY_MN, build_inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def call_single(kind, F, G):
    return br.discriminant(F) if kind == "disc" else br.resultant(F, G)


def test_deg20_bench_batch_pairs_full():
    pairs = [synth.pair_deg20(s) for s in range(256)]
    say("deg20 bench batch: 256 pairs, device memory, plan reuse")
    br.set_plan_cache(True)
    b = br.DeviceBatch([("res", F, G, "y") for F, G in pairs])
    b.run()
    b.run()   # the second call reuses the plans, as every timed step does
    res = b.results()
    assert list(b.status) == [0] * 256
    assert res[0] == load("deg20_res_0.txt")[1]
    for name in nodecheck.names("deg20"):
        rec = nodecheck.case("deg20", name)
        say("  ", name)
        nodecheck.check(res[rec["args"][0]], rec)
    say("  the same batch under the persistent fused schedule")
    try:
        br.set_schedule("fused")
        b.run()
        fused = b.results()
    finally:
        br.set_schedule("staged")
    assert list(b.status) == [0] * 256
    assert fused == res


def check_gcd(R, h):
    """h = gcd(R, R') in Z[x]: it divides both exactly, the cofactors are
    coprime, its content is gcd(cont R, cont R') and its leading coefficient
    is positive; together these fix the normalised gcd."""
    dR = zx.derivative(R)
    qa = zx.exact_div(R, h)
    qb = zx.exact_div(dR, h)
    assert h[-1] > 0
    p = (1 << 61) - 1
    assert qa[-1] % p and qb[-1] % p
    assert gcd_mod_p(qa, qb, p) == [1]
    assert zx.content(h) == zx.content([zx.content(R), zx.content(dR)])


@pytest.mark.parametrize("name", ["curve_deg40_dense", "curve_deg40_g2_hk", "curve_deg40_g2_hk2"])
def test_curve_deg40_full(name):
    rec = nodecheck.case("curve40", name)
    kind, F, _, _ = nodecheck.inputs(rec)
    say(name, "discriminant, D =", rec["D"])
    R = br.discriminant(F)
    nodecheck.check(R, rec)
    say(name, "gcd(R, R')")
    h = br.gcd(R, zx.derivative(R))
    say("  deg gcd =", len(h) - 1)
    check_gcd(R, h)
    if name.endswith("hk2"):
        assert len(h) - 1 >= 1


def test_arrangement_batch_pairs_full():
    curves, pairs = synth.arrangement_batch(0)
    jobs = [("res", curves[i], curves[j], "y") for i, j in pairs]
    recs = [nodecheck.case("arrangement", n) for n in nodecheck.names("arrangement")]
    # the selected pair with the largest prime count has the batch's largest
    Ps = [br.plan(F, G)[1] for _, F, G, _ in jobs]
    assert max(Ps) == max(Ps[rec["args"][0]] for rec in recs), max(Ps)
    say("arrangement batch of", len(jobs), "pairs, prime counts up to", max(Ps))
    b = br.DeviceBatch(jobs)
    try:
        br.set_schedule("staged")
        b.run()
        staged = b.results()
        assert list(b.status) == [0] * len(jobs)
        br.set_schedule("fused")
        b.run()
        fused = b.results()
    finally:
        br.set_schedule("staged")
    assert fused == staged
    for rec in recs:
        k = rec["args"][0]
        say("  ", rec["name"], rec.get("note", ""), "P =", Ps[k])
        nodecheck.check(staged[k], rec)
        assert br.resultant(*jobs[k][1:3]) == staged[k]


def test_serving_requests_above_128_primes_full():
    recs = [nodecheck.case("serving", n) for n in nodecheck.names("serving")]
    stream = synth.poisson_requests(0, n=2000)
    sel = [rec["args"][0] for rec in recs]
    for rec in recs:
        kind, F, G, _ = nodecheck.inputs(rec)
        assert br.plan(F, G, kind=kind)[1] > 128
    # the selected requests arrive in a mix with the first 40 requests of the stream
    order = sorted(set(range(40)) | set(sel))
    say("server: %d requests, selected %s" % (len(order), sel))
    with br.Server(hbm_budget_bytes=4 << 30, max_slots=32) as srv:
        tickets = {i: srv.submit(stream[i]["kind"], stream[i]["f"], stream[i]["g"]) for i in order}
        served = {i: srv.wait(t)[0] for i, t in tickets.items()}
    for rec in recs:
        kind, F, G, _ = nodecheck.inputs(rec)
        i = rec["args"][0]
        say("  ", rec["name"], rec.get("note", ""), kind)
        nodecheck.check(served[i], rec)
        assert call_single(kind, F, G) == served[i]
    for i in order[:12]:
        r = stream[i]
        assert served[i] == call_single(r["kind"], r["f"], r["g"]), i


@pytest.mark.parametrize("mn", CAPACITY_MN)
def test_capacity_boundaries_full(mn):
    rec = nodecheck.case("capacity", "capacity_%d_%d" % mn)
    _, F, G, _ = nodecheck.inputs(rec)
    jobs = [("res", F, G, "y")] * 2 + [("res",) + synth.pair_deg6(1) + ("y",)]
    say("capacity boundary", mn)
    try:
        br.set_eval_kernel("lds")
        lds, st_l = br.resultant_batch(jobs)
        br.set_eval_kernel("auto")
        reg, st_r = br.resultant_batch(jobs)
        br.set_schedule("fused")
        fus, st_f = br.resultant_batch(jobs)
    finally:
        br.set_eval_kernel("auto")
        br.set_schedule("staged")
    assert st_l == st_r == st_f == [0, 0, 0]
    nodecheck.check(reg[0], rec)
    assert lds == reg == fus and reg[1] == reg[0] == br.resultant(F, G)


# ---------------------------------------------------------------------------
# more than 128 primes: Garner digits and limb kernels instead of the
# explicit CRT; small y-degree keeps the oracle's Bareiss cheap

BIG = [(5, 6, 5, 6, 400), (4, 8, 4, 8, 500), (6, 4, 5, 4, 360), (3, 10, 3, 10, 700)]


@pytest.mark.parametrize("i", range(len(BIG)))
def test_more_than_128_primes_single_call(i):
    F, G = synth.random_rect(1300 + i, *BIG[i])
    D, P, _ = br.plan(F, G)
    say("P > 128 single call", BIG[i], "D", D, "P", P)
    assert P > 128
    assert br.resultant(F, G) == resultant_y(F, G)


def test_more_than_128_primes_mixed_batches():
    big = [synth.random_rect(1300 + i, *BIG[i]) for i in range(len(BIG))]
    small = [synth.pair_deg6(i % 4) for i in range(6)]
    disc = synth.random_rect(1400, 5, 5, 1, 1, 520)[0]
    jobs = [("res", F, G, "y") for F, G in big] + [("res", F, G, "y") for F, G in small]
    jobs += [("disc", disc, None, "y"), ("res", big[0][1], big[0][0], "y")]
    refs = [resultant_y(F, G) for _, F, G, _ in jobs[:-2]]
    refs += [resultant_y(disc, bi_diff_y(disc)), resultant_y(big[0][1], big[0][0])]
    assert br.plan(disc, kind="disc")[1] > 128
    say("mixed batch with P > 128 jobs:", len(jobs))
    res, st = br.resultant_batch(jobs)
    assert st == [0] * len(jobs)
    assert res == refs
    # the same jobs among enough deg-20 pairs that the batch has >= 16384 output coefficients
    filler = [("res",) + synth.pair_deg20(s) + ("y",) for s in range(42)]
    res2, st2 = br.resultant_batch(jobs + filler)
    assert st2 == [0] * len(jobs + filler)
    assert res2[:len(jobs)] == refs
    assert res2[len(jobs)] == load("deg20_res_0.txt")[1]
    # the persistent fused schedule takes the same Garner route
    try:
        br.set_schedule("fused")
        res3, st3 = br.resultant_batch(jobs + filler)
    finally:
        br.set_schedule("staged")
    assert st3 == st2 and res3 == res2
    b = br.DeviceBatch(jobs)
    b.run()
    assert b.results() == refs


def test_large_fused_batch_of_mixed_shapes():
    # the persistent fused schedule on two shapes (no matrix-core group: the
    # interpolation per (job, prime)), reconstructed by the explicit CRT
    jobs = [("res",) + synth.pair_deg20(s) + ("y",) for s in range(42)]
    jobs += [("res",) + synth.pair_deg6(i) + ("y",) for i in range(4)]
    say("fused batch of", len(jobs))
    try:
        br.set_schedule("fused")
        res, st = br.resultant_batch(jobs)
    finally:
        br.set_schedule("staged")
    assert st == [0] * len(jobs)
    assert res[0] == load("deg20_res_0.txt")[1]
    for i in range(4):
        assert res[42 + i] == load("deg6_res_%d.txt" % i)[1]
    rec = nodecheck.case("deg20", "deg20_pair_37")
    nodecheck.check(res[37], rec)
