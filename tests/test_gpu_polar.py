"""Q = res(f_x, f_y; y), the resultant of the fiber bound n_alpha^+ (Section
3.2.2, "Computation of n_alpha^+"), through every entry point that takes the
polar kind, against the oracle (oracle.subresultants.polar_resultant_y).

* small curves of every shape (random dense, multi-limb coefficients, var = x,
  a row-degree drop of f_x, f_x = 0, m_y = 1) in full;
* the degree-40 curves and the largest arrangement curve at full size through
  the node digests the oracle wrote (tests/nodecheck.py), as single calls;
* batches that mix the three kinds, with batched == single bit for bit;
* the server and the allocation-free entry point.
"""

import random

import pytest

import paper_1201_1548_amd as br
from oracle.resultant import bi_transpose, bi_trim
from oracle.subresultants import polar_resultant_y
from paper_1201_1548_amd import synth
from tests import nodecheck

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rand_curve(rng, t, bits, ydeg=None):
    ydeg = t if ydeg is None else ydeg
    F = [[rng.randint(-(1 << (bits - 1)), (1 << (bits - 1)) - 1) for _ in range(t - j + 1)] for j in range(ydeg + 1)]
    F[-1][0] = F[-1][0] or 1
    return F


@pytest.mark.parametrize("seed", range(6))
def test_polar_small_curves(seed):
    rng = random.Random(seed)
    t = rng.randint(2, 8)
    bits = rng.choice([4, 16, 31, 70, 130])
    F = rand_curve(rng, t, bits)
    say("seed", seed, "tdeg", t, "bits", bits)
    assert br.polar_resultant(F) == polar_resultant_y(F)


def test_polar_var_x():
    rng = random.Random(11)
    F = rand_curve(rng, 5, 20)
    # res(f_y, f_x; x) is Q of the transposed curve
    assert br.polar_resultant(F, var="x") == polar_resultant_y(bi_transpose(F))


def test_polar_edge_cases():
    # f_x = 0 (f free of x): Q = 0
    assert br.polar_resultant([[3], [0], [5]]) == []
    # m_y = 1: f = f_1(x) y + f_0(x), f_y = f_1 of y-degree 0
    F = [[1, 2, 3], [4, -5]]
    assert br.polar_resultant(F) == polar_resultant_y(F)
    # f_x of lower y-degree than f (the top row constant in x)
    F = [[1, 2, 3, 4], [5, -6, 7], [8, 9], [10]]
    assert br.polar_resultant(F) == polar_resultant_y(F)
    # m_y = 0 is rejected like the discriminant
    with pytest.raises(br.BiresError) as e:
        br.polar_resultant([[1, 2, 3]])
    assert e.value.code == -1


@pytest.mark.parametrize("name", nodecheck.names("polar"))
def test_polar_full_size_against_oracle_nodes(name):
    rec = nodecheck.case("polar", name)
    kind, F, _, _ = nodecheck.inputs(rec)
    say(name, "D =", rec["D"])
    Q = br.polar_resultant(F)
    nodecheck.check(Q, rec)


def test_polar_in_mixed_batch():
    rng = random.Random(5)
    jobs = []
    for k in range(12):
        F = rand_curve(rng, rng.randint(3, 9), rng.choice([8, 32, 64]))
        G = rand_curve(rng, rng.randint(2, 7), 16)
        jobs.append((("res", "disc", "polar")[k % 3], F, G if k % 3 == 0 else None, "y"))
    res, status = br.resultant_batch(jobs)
    assert status == [0] * len(jobs)
    for (kind, F, G, _), r in zip(jobs, res):
        if kind == "polar":
            assert r == polar_resultant_y(F)
            assert r == br.polar_resultant(F)
        elif kind == "disc":
            assert r == br.discriminant(F)
        else:
            assert r == br.resultant(F, G)


def test_polar_device_batch_matches_plain():
    import torch
    curves = [synth.curve_deg40(20 + i, tdeg=14, bits=24) for i in range(40)]
    b = br.DeviceBatch([("polar", F, None, "y") for F in curves])
    b.run()
    torch.cuda.synchronize()
    got = b.results()
    b.run_each()
    torch.cuda.synchronize()
    assert b.results() == got
    assert got[0] == polar_resultant_y(curves[0])


def test_polar_through_server_and_noalloc():
    rng = random.Random(8)
    curves = [rand_curve(rng, rng.randint(3, 7), 40) for _ in range(6)]
    with br.Server(hbm_budget_bytes=1 << 30, max_slots=8) as srv:
        tickets = [srv.submit("polar", F) for F in curves]
        outs = [srv.wait(t)[0] for t in tickets]
    br.init()
    for F, q in zip(curves, outs):
        want = polar_resultant_y(F)
        assert q == want
        assert br.resultant_noalloc(F, kind="polar") == want
