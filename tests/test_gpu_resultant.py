"""Parity of the HIP path (through the C ABI) with the oracle: bit-exact.

Stage parity: the univariate resultants the kernel produces at (prime p, point a)
equal R(a) mod p of the oracle's R.  End-to-end parity: the reconstructed
coefficients equal the oracle's (or the stored golden values the oracle wrote).
Covers several tiles and ragged tails (points not a multiple of 64, residue
counts not a multiple of the tile), degree drops at a = 0, zero inputs,
y-free inputs, res_x, the discriminant, batches and device-memory buffers.
"""

import os
import random

import pytest

import paper_1201_1548_amd as br
from oracle import zx
from oracle.closed_forms import product_discriminant, product_pair
from oracle.resultant import discriminant_y, resultant_at, resultant_x, resultant_y
from paper_1201_1548_amd import synth
from tests.golden.make_golden import input_digest, load

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)


def test_stage_values_deg6():
    F, G = synth.pair_deg6(0)
    say("stage values deg6 instance 0")
    _, R = load("deg6_res_0.txt")
    ps, vals = br.debug_values(F, G)
    assert vals.shape == (len(ps), 37)
    for k, p in enumerate(ps):
        for a in range(vals.shape[1]):
            assert int(vals[k, a]) == zx.evaluate(R, a) % p, (k, a)


@pytest.mark.parametrize("inst", range(4))
def test_deg6_bit_exact(inst):
    F, G = synth.pair_deg6(inst)
    say("deg6 instance", inst)
    digest, R = load("deg6_res_%d.txt" % inst)
    assert digest == input_digest(F, G)
    assert br.resultant(F, G) == R


SHAPES = [  # (ydeg f, xdeg f, ydeg g, xdeg g, bits)
    (1, 3, 1, 2, 16), (3, 1, 2, 4, 40), (4, 4, 3, 5, 31), (2, 6, 5, 2, 70),
    (5, 3, 5, 3, 12), (6, 2, 1, 7, 100), (1, 0, 4, 3, 20), (7, 3, 6, 2, 33),
]


@pytest.mark.parametrize("i", range(len(SHAPES)))
def test_random_shapes(i):
    a, b, c, d, bits = SHAPES[i]
    F, G = synth.random_rect(100 + i, a, b, c, d, bits)
    say("random shape", SHAPES[i])
    assert br.resultant(F, G) == resultant_y(F, G)


@pytest.mark.parametrize("i", range(4))
def test_random_shapes_x(i):
    a, b, c, d, bits = SHAPES[i]
    F, G = synth.random_rect(200 + i, a, b, c, d, bits)
    say("res_x shape", SHAPES[i])
    assert br.resultant(F, G, var="x") == resultant_x(F, G)


@pytest.mark.parametrize("seed", range(4))
def test_discriminant_random(seed):
    F, _ = synth.random_rect(300 + seed, 2 + seed, 3, 1, 1, 24 + 10 * seed)
    say("discriminant seed", seed)
    assert br.discriminant(F) == discriminant_y(F)


def test_discriminant_closed_form_and_repeated_root():
    rng = random.Random(5)
    roots = [[rng.randint(-9, 9) for _ in range(3)] for _ in range(5)]
    f, R = product_discriminant([3, 0, 1], roots)
    say("discriminant closed form")
    assert br.discriminant(f) == R
    f2, R2 = product_discriminant([1, 1], [[1, 2], [1, 2], [0, 5]])
    assert R2 == [] and br.discriminant(f2) == []


def test_sparse_inputs_with_zero_rows():
    F, G = synth.random_rect(400, 5, 4, 4, 5, 30, zero_frac=0.6)
    say("sparse inputs")
    assert br.resultant(F, G) == resultant_y(F, G)


def test_degree_drops_at_zero():
    # lc_y f = x (vanishes at a = 0), lc_y g = x + 1: formal-degree rule for f
    F = [[1, 2, 3], [4, 0, 5], [0, 1]]
    G = [[2, -1], [7, 3, 1], [1, 1]]
    say("degree drops")
    assert br.resultant(F, G) == resultant_y(F, G)
    # both leading coefficients vanish at 0
    G2 = [[2, -1], [7, 3, 1], [0, 2]]
    assert br.resultant(F, G2) == resultant_y(F, G2)
    # lc of g vanishes at 0 only
    assert br.resultant(G, F) == resultant_y(G, F)
    # f(0, y) identically zero
    F0 = [[0, 1], [0, 2], [0, 0, 3]]
    assert br.resultant(F0, G) == resultant_y(F0, G)


def test_edge_conventions():
    say("edge conventions")
    G = [[1, 2], [0, 1], [5]]
    assert br.resultant([[3, -1, 2]], G) == resultant_y([[3, -1, 2]], G)   # m_y = 0
    assert br.resultant(G, [[3, -1, 2]]) == resultant_y(G, [[3, -1, 2]])   # n_y = 0
    assert br.resultant([[3, 1]], [[7, 2]]) == [1]                          # empty determinant
    assert br.resultant([[0, 0]], G) == [] and br.resultant(G, []) == []    # zero input
    assert br.resultant([[0], [0], [0], [4]], [[1], [1]]) == resultant_y([[0], [0], [0], [4]], [[1], [1]])
    with pytest.raises(br.BiresError):
        br.discriminant([[1, 2, 3]])


def test_closed_form_product_pair():
    rng = random.Random(9)
    A = [rng.randint(-5, 5) for _ in range(3)]
    B = [1, rng.randint(-5, 5)]
    a = [[rng.randint(-99, 99) for _ in range(3)] for _ in range(6)]
    b = [[rng.randint(-99, 99) for _ in range(2)] for _ in range(5)]
    f, g, R = product_pair(A, a, B, b)
    say("closed form product pair")
    assert br.resultant(f, g) == R
    b[2] = a[4]                          # common root: R = 0
    f, g, R = product_pair(A, a, B, b)
    assert R == [] and br.resultant(f, g) == []


def test_batch_equals_single_and_oracle():
    jobs = []
    for i in range(6):
        a, b, c, d, bits = SHAPES[i]
        F, G = synth.random_rect(500 + i, a, b, c, d, bits)
        jobs.append(("res", F, G, "y"))
    F, G = synth.pair_deg6(1)
    jobs.append(("res", F, G, "y"))
    jobs.append(("res", F, G, "x"))
    jobs.append(("disc", F, None, "y"))
    jobs.append(("res", [[0]], G, "y"))
    jobs.append(("res", [[3, 1]], [[7, 2]], "y"))
    say("batch of", len(jobs))
    res, st = br.resultant_batch(jobs)
    assert st == [0] * len(jobs)
    for (kind, F, G, var), R in zip(jobs, res):
        if kind == "disc":
            ref = discriminant_y(F)
            assert br.discriminant(F) == R
        else:
            ref = resultant_y(F, G) if var == "y" else resultant_x(F, G)
            assert br.resultant(F, G, var) == R
        assert R == ref


def test_batch_reports_per_job_errors():
    F, G = synth.pair_deg6(0)
    res, st = br.resultant_batch([("res", F, G, "y"), ("disc", [[1, 2]], None, "y"), ("res", G, F, "y")])
    assert st[0] == 0 and st[2] == 0 and st[1] == -1
    assert res[0] == resultant_y(F, G) and res[2] == resultant_y(G, F)


def test_device_memory_batch():
    F, G = synth.pair_deg6(2)
    H, K = synth.random_rect(600, 3, 4, 4, 2, 50)
    jobs = [("res", F, G, "y"), ("res", H, K, "x"), ("disc", H, None, "y"), ("res", [[5]], [[1, 1]], "y")]
    say("device-memory batch")
    b = br.DeviceBatch(jobs)
    b.run()
    out = b.results()
    assert out[0] == resultant_y(F, G)
    assert out[1] == resultant_x(H, K)
    assert out[2] == discriminant_y(H)
    assert out[3] == [1]
    b.run_each()
    assert b.results() == out


def test_deg20_spot_values():
    F, G = synth.pair_deg20(0)
    say("deg20 spot values")
    R = br.resultant(F, G)
    assert len(R) - 1 <= 400
    for a in (0, 1, -1, 2, 12345):
        assert zx.evaluate(R, a) == resultant_at(F, G, a), a


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "deg20_res_0.txt")),
                    reason="degree-20 golden file not generated")
def test_deg20_golden_bit_exact():
    F, G = synth.pair_deg20(0)
    say("deg20 golden")
    digest, R = load("deg20_res_0.txt")
    assert digest == input_digest(F, G)
    assert br.resultant(F, G) == R


def _mixed_jobs():
    jobs = []
    for i in range(8):
        a, b, c, d, bits = SHAPES[i]
        F, G = synth.random_rect(700 + i, a, b, c, d, bits)
        jobs.append(("res", F, G, "y" if i % 3 else "x"))
    for i in range(24):
        F, G = synth.pair_deg6(i % 4)
        jobs.append(("res", F, G, "y"))
    F, G = synth.pair_deg20(3)
    jobs.append(("res", F, G, "y"))
    H, _ = synth.random_rect(800, 5, 3, 1, 1, 40)
    jobs += [("disc", H, None, "y"), ("res", [[0]], G, "y"), ("res", [[3, 1]], [[7, 2]], "y"),
             ("disc", [[1, 2]], None, "y")]
    return jobs


@pytest.mark.parametrize("schedule", ["fused", "auto"])
def test_fused_schedule_matches_staged(schedule):
    jobs = _mixed_jobs()
    say("schedule", schedule, "jobs", len(jobs))
    br.set_schedule("staged")
    ref, st_ref = br.resultant_batch(jobs)
    try:
        br.set_schedule(schedule)
        got, st_got = br.resultant_batch(jobs)
        b = br.DeviceBatch([j for j in jobs if not (j[0] == "disc" and len(j[1]) < 2)])
        b.run()
        dev = b.results()
    finally:
        br.set_schedule("staged")
    assert st_got == st_ref and st_ref[-1] == -1 and st_ref.count(0) == len(jobs) - 1
    assert got == ref
    assert dev == [r for r, j in zip(ref, jobs) if not (j[0] == "disc" and len(j[1]) < 2)]
    for (kind, F, G, var), R in list(zip(jobs, ref))[:12]:
        if kind == "res":
            assert R == (resultant_y(F, G) if var == "y" else resultant_x(F, G))


def test_fused_batches_in_flight_on_two_streams():
    # two persistent fused launches at once on two streams: neither holds the
    # whole device, so each launch's stages must drain with the blocks it has
    # (tasks are claimed, a stage ends on its count of finished tasks); one
    # batch takes the matrix-core interpolation, the other the per-(job, prime)
    # one
    import torch
    jobs_a = [("res",) + synth.pair_deg20(s) + ("y",) for s in range(256)]
    jobs_b = [("res",) + synth.pair_deg6(i % 4) + ("y",) for i in range(40)]
    say("fused batches on two streams", len(jobs_a), len(jobs_b))
    a, b = br.DeviceBatch(jobs_a), br.DeviceBatch(jobs_b)
    br.set_schedule("staged")
    a.run()
    b.run()
    ref_a, ref_b = a.results(), b.results()
    assert ref_a[0] == load("deg20_res_0.txt")[1]
    assert ref_b[:4] == [load("deg6_res_%d.txt" % i)[1] for i in range(4)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    try:
        br.set_schedule("fused")
        for rep in range(3):
            a.run_async(s1)
            b.run_async(s2)
            a.wait()
            b.wait()
            assert a.results() == ref_a, rep
            assert b.results() == ref_b, rep
    finally:
        br.set_schedule("staged")


def test_fused_matrix_core_group_above_48_primes():
    # 32 copies of a pair with 200-bit coefficients (D = 73, P = 80): the
    # fused launch with the matrix-core interpolation group and the CRT for up
    # to 128 primes, against the oracle's Bareiss value and the staged schedule
    F, G = synth.random_rect(2100, 6, 6, 6, 6, 200)
    D, P, _ = br.plan(F, G)
    assert 48 < P <= 128, P
    jobs = [("res", F, G, "y")] * 32
    say("fused group of 32, D", D, "P", P)
    ref = resultant_y(F, G)
    b = br.DeviceBatch(jobs)
    try:
        br.set_schedule("staged")
        b.run()
        staged = b.results()
        br.set_schedule("fused")
        b.run()
        fused = b.results()
    finally:
        br.set_schedule("staged")
    assert staged == [ref] * 32
    assert fused == staged


def test_autotune_keeps_results():
    jobs = [("res",) + synth.pair_deg6(i % 4) + ("y",) for i in range(16)]
    say("autotune")
    b = br.DeviceBatch(jobs)
    choice = b.autotune(reps=1)
    assert choice in ("staged", "fused", "schur")
    out = b.results()
    assert out == [resultant_y(F, G) for _, F, G, _ in jobs]
    br.set_schedule("auto")
    b.run()
    assert b.results() == out


def test_large_batch_mixed_shapes():
    # 50 jobs of two shapes (>= 16384 output coefficients, at most 48 primes):
    # the staged schedule reconstructs them with the explicit CRT on the
    # matrix cores, like single calls
    jobs = [("res",) + synth.pair_deg20(i) + ("y",) for i in range(40)]
    jobs += [("res",) + synth.pair_deg6(i % 4) + ("y",) for i in range(10)]
    say("large batch", len(jobs))
    res, st = br.resultant_batch(jobs)
    assert st == [0] * len(jobs)
    _, R0 = load("deg20_res_0.txt")
    assert res[0] == R0
    for i in range(10):
        assert res[40 + i] == load("deg6_res_%d.txt" % (i % 4))[1]
    for i in (1, 17, 39):
        assert res[i] == br.resultant(*synth.pair_deg20(i))
        for a in (3, -7):
            assert zx.evaluate(res[i], a) == resultant_at(*synth.pair_deg20(i), a)


def test_shared_shape_batch_matrix_core_interpolation():
    # >= 32 jobs with the same point and prime counts interpolate as int8
    # matrix-core products with the inverse Vandermonde matrix; single calls
    # use the per-job interpolation kernel
    pairs = [synth.pair_deg20(i) for i in range(36)]
    D, P, _ = br.plan(*pairs[0])
    assert all(br.plan(F, G)[:2] == (D, P) for F, G in pairs)
    say("shared-shape batch", len(pairs), D, P)
    res, st = br.resultant_batch([("res", F, G, "y") for F, G in pairs])
    assert st == [0] * len(pairs)
    assert res[0] == load("deg20_res_0.txt")[1]
    for i, (F, G) in enumerate(pairs):
        assert res[i] == br.resultant(F, G), i
    for i in (5, 35):
        assert zx.evaluate(res[i], 11) == resultant_at(*pairs[i], 11)


@pytest.mark.parametrize("n", [32, 33, 97])
def test_matrix_core_interpolation_block_edges(n):
    # the matrix-core interpolation runs four-wave blocks over 64 x 64 blocks
    # of the coefficient matrix: 32 jobs leave a block's second column tile
    # past the matrix, 33 and 97 jobs leave part of the last column tile past
    # the group, and the deg-6 point count fills one row-tile pair exactly
    # (deg-6 pairs 0 and 3 share D = 37 and P = 5, which the path needs)
    idx = [(0, 3)[i % 2] for i in range(n)]
    jobs = [("res",) + synth.pair_deg6(j) + ("y",) for j in idx]
    assert len({br.plan(F, G)[:2] for _, F, G, _ in jobs}) == 1
    say("deg6 batch", n)
    res, st = br.resultant_batch(jobs)
    assert st == [0] * n
    for i, j in enumerate(idx):
        assert res[i] == load("deg6_res_%d.txt" % j)[1], i


@pytest.mark.parametrize("kernel", ["auto", "lds", "schur"])
def test_matrix_core_interpolation_from_every_evaluation_kernel(kernel):
    # in a batch of >= 32 jobs sharing D and P the evaluation kernels write the
    # values straight into the interpolation's digit planes: the register
    # kernel, the LDS kernel and the Schur kernel each against the oracle
    pairs = [synth.pair_deg20(i) for i in range(34)]
    say("deg20 batch, evaluation kernel", kernel)
    br.set_eval_kernel(kernel)
    try:
        res, st = br.resultant_batch([("res", F, G, "y") for F, G in pairs])
    finally:
        br.set_eval_kernel("auto")
    assert st == [0] * len(pairs)
    assert res[0] == load("deg20_res_0.txt")[1]
    for i in (1, 20, 33):
        for x in (2, -9):
            assert zx.evaluate(res[i], x) == resultant_at(*pairs[i], x), (i, x)


def test_deg20_full_batch_in_the_bench_configuration():
    # the timed workload itself: 256 dense total-degree-20 pairs as device-memory batches
    # (plan reuse on), synchronous and with two batches in flight; pair 0
    # equals the stored oracle value, every pair the single call, sampled
    # pairs the oracle's determinant at nodes, every repeat the first run
    pairs = [synth.pair_deg20(s) for s in range(256)]
    jobs = [("res", F, G, "y") for F, G in pairs]
    say("deg20 full batch", len(jobs))
    br.set_plan_cache(True)
    a, b = br.DeviceBatch(jobs), br.DeviceBatch(jobs)
    a.run()
    ref = a.results()
    assert list(a.status) == [0] * len(jobs)
    assert ref[0] == load("deg20_res_0.txt")[1]
    for i, (F, G) in enumerate(pairs):
        assert ref[i] == br.resultant(F, G), i
    for i in (1, 97, 255):
        for x in (5, -3):
            assert zx.evaluate(ref[i], x) == resultant_at(*pairs[i], x), (i, x)
    for _ in range(3):
        a.run()
        assert a.results() == ref
    prev = None
    for k in range(6):
        cur = (a, b)[k % 2]
        cur.run_async()
        if prev is not None:
            prev.wait()
            assert prev.results() == ref, k
        prev = cur
    prev.wait()
    assert prev.results() == ref


@pytest.mark.parametrize("schedule", ["staged", "fused"])
def test_graph_replay_matches_eager(schedule):
    # batched calls replayed from captured HIP graphs: every replay, with eager
    # work and synchronisations between replays and another batch's graph in
    # between, equals the eagerly issued result
    import torch
    jobs = [j for j in _mixed_jobs() if not (j[0] == "disc" and len(j[1]) < 2)]
    say("graph replay", schedule, len(jobs))
    br.set_schedule(schedule)
    try:
        b = br.DeviceBatch(jobs)
        b.run()
        eager = b.results()
        other = br.DeviceBatch([("res",) + synth.pair_deg6(i % 4) + ("y",) for i in range(6)])
        other.run()
        eager_other = other.results()
        host_ref = br.resultant_batch(jobs)
        br.set_graphs(True)
        c0, r0 = br.graph_stats()
        for rep in range(4):
            for t in b.out_tensors:
                t.fill_(-1)
            torch.cuda.synchronize()
            b.run()
            assert b.results() == eager, rep
            if rep == 1:
                for t in other.out_tensors:
                    t.zero_()
                other.run()
                assert other.results() == eager_other
            assert br.resultant_batch(jobs) == host_ref, rep
        c1, r1 = br.graph_stats()
        say("graphs captured", c1 - c0, "replayed", r1 - r0)
        assert r1 - r0 >= 4 and c1 - c0 >= 2
    finally:
        br.set_graphs(False)
        br.set_schedule("staged")
    assert eager[:len(jobs)] == host_ref[0]


def test_register_and_lds_evaluation_kernels_agree():
    # the register-array kernel (with its fallback queue) and the general LDS
    # kernel give the same results on generic jobs and on jobs whose leading
    # coefficients vanish at some points or whose remainder sequences are not
    # normal (every block of those falls back)
    jobs = [j for j in _mixed_jobs() if not (j[0] == "disc" and len(j[1]) < 2)]
    jobs += [("res",) + synth.pair_deg20(i) + ("y",) for i in range(3)]
    # lc_y(f) = x - 5 vanishes at a = 5; in the second pair lc_y(g) = x^2
    # vanishes at a = 0 and the first remainder's y-coefficient
    # x^3 - 3x - 2 = (x + 1)^2 (x - 2) at a = 2
    jobs += [("res", [[2], [3, 7], [-5, 1]], [[1, 1, 4], [0, 2]], "y"),
             ("res", [[7, 0, 1], [0, 1], [1]], [[1], [2, 3], [0, 0, 1]], "y")]
    say("register vs lds kernels", len(jobs))
    try:
        br.set_eval_kernel("lds")
        ref, st_ref = br.resultant_batch(jobs)
        br.set_eval_kernel("auto")
        got, st_got = br.resultant_batch(jobs)
        single = [br.resultant(F, G, var) if k == "res" else None for k, F, G, var in jobs[-5:]]
    finally:
        br.set_eval_kernel("auto")
    assert st_got == st_ref
    assert got == ref
    assert got[-5:-2] == single[:3]
    for (kind, F, G, var), R in list(zip(jobs, got))[-2:]:
        assert R == resultant_y(F, G)


def test_async_batches_overlap_and_match():
    # two device batches alternately in flight (planned and queued by the caller);
    # every result equals the synchronous call's, also with the caller's
    # stream still busy writing the inputs when the batch is queued
    import torch
    jobs_a = [j for j in _mixed_jobs() if not (j[0] == "disc" and len(j[1]) < 2)]
    jobs_b = [("res",) + synth.pair_deg6(i % 4) + ("y",) for i in range(20)]
    say("async batches", len(jobs_a), len(jobs_b))
    a, b = br.DeviceBatch(jobs_a), br.DeviceBatch(jobs_b)
    a.run()
    ref_a = a.results()
    b.run()
    ref_b = b.results()
    for rep in range(3):
        for t in a.out_tensors + b.out_tensors:
            t.fill_(7)
        torch.cuda.synchronize()  # no stream given: the buffers must be settled
        a.run_async()
        b.run_async()
        a.wait()
        b.wait()
        assert a.results() == ref_a, rep
        assert b.results() == ref_b, rep
    # inputs rewritten on a side stream right before the submission: the
    # batch must see the new values (zeroed f rows give the zero resultant)
    s = torch.cuda.Stream()
    f0 = a.inputs[0][0]
    saved = f0.tensor.clone()
    with torch.cuda.stream(s):
        torch.cuda._sleep(2000000)
        f0.tensor.zero_()
        a.run_async(stream=s)
    a.wait()
    got = a.results()
    assert got[0] == []
    assert got[1:] == ref_a[1:]
    f0.tensor.copy_(saved)
    torch.cuda.synchronize()
    bad = br.lib().bires_batch_wait(123456789)
    assert bad != 0


def test_plan_reuse_is_checked_on_the_device():
    # repeated device batches reuse the previous plans; a changed input whose
    # row statistics stay the same keeps them (and its new results), one whose
    # statistics change is caught by the device check and rerun
    import torch
    pairs = [synth.pair_deg6(i % 4) for i in range(12)] + [synth.pair_deg20(5)]
    jobs = [("res", F, G, "y") for F, G in pairs]
    say("plan reuse", len(jobs))
    br.set_plan_cache(True)
    b = br.DeviceBatch(jobs)
    ref = [load("deg6_res_%d.txt" % (i % 4))[1] for i in range(12)] + [br.resultant(*pairs[-1])]
    h0, m0 = br.plan_cache_stats()
    for _ in range(4):
        b.run()
        assert b.results() == ref
    h1, m1 = br.plan_cache_stats()
    assert h1 - h0 >= 2 and m1 == m0
    # negate f's coefficient of x^1 y^0 in job 0: same magnitudes, same statistics
    F0 = [list(r) for r in pairs[0][0]]
    t = b.inputs[0][0].tensor
    assert b.inputs[0][0].shape[2] == 1  # one 32-bit limb per coefficient
    F0[0][1] = -F0[0][1]
    t.view(-1)[1] = -int(t.view(-1)[1].item())
    torch.cuda.synchronize()
    b.run()
    got = b.results()
    assert got[0] == resultant_y(F0, pairs[0][1])
    assert got[1:] == ref[1:]
    h2, m2 = br.plan_cache_stats()
    assert h2 == h1 + 1 and m2 == m1
    # a coefficient far larger than before: new statistics, caught and rerun
    F0[0][1] = 1 << 29
    t.view(-1)[1] = 1 << 29
    torch.cuda.synchronize()
    b.run()
    got = b.results()
    assert got[0] == resultant_y(F0, pairs[0][1])
    assert got[1:] == ref[1:]
    h3, m3 = br.plan_cache_stats()
    assert m3 == m2 + 1
    br.set_plan_cache(False)
    b.run()
    assert b.results()[0] == got[0]
    br.set_plan_cache(True)


def test_plan_reuse_with_alternating_batches_in_flight():
    # two batches of the same shapes in separate buffers, two calls in flight:
    # both reuse the plans (addresses are not part of the key); a statistics
    # change in one of them while the other is in flight is caught and rerun
    import torch
    pairs = [synth.pair_deg6(i % 4) for i in range(12)] + [synth.pair_deg20(5)]
    jobs = [("res", F, G, "y") for F, G in pairs]
    say("alternating plan reuse", len(jobs))
    br.set_plan_cache(True)
    a, b = br.DeviceBatch(jobs), br.DeviceBatch(jobs)
    ref = [load("deg6_res_%d.txt" % (i % 4))[1] for i in range(12)] + [br.resultant(*pairs[-1])]
    for x in (a, b):
        x.run()
        assert x.results() == ref
    h0, m0 = br.plan_cache_stats()
    prev = None
    for k in range(8):
        x = (a, b)[k % 2]
        x.run_async()
        if prev is not None:
            prev.wait()
            assert prev.results() == ref, k
        prev = x
    prev.wait()
    assert prev.results() == ref
    h1, m1 = br.plan_cache_stats()
    assert h1 - h0 >= 6 and m1 == m0
    # b's job 0 gets a much larger coefficient while a is in flight
    F0 = [list(r) for r in pairs[0][0]]
    F0[0][1] = 1 << 29
    t = b.inputs[0][0].tensor
    assert b.inputs[0][0].shape[2] == 1
    a.run_async()
    t.view(-1)[1] = 1 << 29
    torch.cuda.synchronize()
    b.run_async()
    a.wait()
    b.wait()
    assert a.results() == ref
    got = b.results()
    assert got[0] == resultant_y(F0, pairs[0][1])
    assert got[1:] == ref[1:]
    h2, m2 = br.plan_cache_stats()
    assert m2 == m1 + 1


@pytest.mark.parametrize("mn", [(23, 9), (9, 23), (24, 4), (31, 31), (31, 2), (32, 6), (5, 0), (0, 7), (1, 1)])
def test_evaluation_kernel_capacity_boundaries(mn):
    # jobs on both sides of each routing boundary (capacity 24, capacity 32,
    # LDS kernel, min(m, n) = 0): register and LDS kernels, batched and single
    # calls agree, and the result matches the oracle's determinant at nodes
    m, n = mn
    F, G = synth.random_rect(900 + 37 * m + n, m, 2, n, 1, 20)
    jobs = [("res", F, G, "y")] * 2 + [("res",) + synth.pair_deg6(1) + ("y",)]
    say("capacity boundary", m, n)
    try:
        br.set_eval_kernel("lds")
        ref, st_ref = br.resultant_batch(jobs)
        br.set_eval_kernel("auto")
        got, st_got = br.resultant_batch(jobs)
    finally:
        br.set_eval_kernel("auto")
    assert st_got == st_ref == [0, 0, 0]
    assert got == ref
    assert got[0] == got[1] == br.resultant(F, G)
    for a in (0, 1, -3, 7):
        assert zx.evaluate(got[0], a) == resultant_at(F, G, a), a
