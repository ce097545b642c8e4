"""The Schur elimination on the displacement generators (k_schur, one wave per
(prime, point) instance, 1 or 2 generator rows per lane) against the oracle.

* every (prime, point) value of small pairs against the oracle's determinant
  of the specialised Sylvester matrix mod p (stage view), with and without
  vanishing leading coefficients (the fallback to Euclid, counted);
* full results through the Schur schedule against the oracle's node digests:
  bench-batch pairs (r = 40), the capacity-boundary jobs, and the degree-40
  discriminants (r = 79: two generator rows per lane);
* r = 120 (two rows per lane, the top of the range) against Euclid's results
  and sampled oracle values;
* mixed batches with jobs outside the Schur range (min(m, n) = 0, r > 128);
* the autotuner over staged, fused and Schur.
"""

import random

import pytest

import paper_1201_1548_amd as br
from oracle import zx
from oracle.resultant import resultant_at_mod
from paper_1201_1548_amd import synth
from tests import nodecheck
from tests.golden.make_golden import load

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


class eval_kernel:
    def __init__(self, name):
        self.name = name

    def __enter__(self):
        br.set_eval_kernel(self.name)

    def __exit__(self, *exc):
        br.set_eval_kernel("auto")


class schedule:
    def __init__(self, name):
        self.name = name

    def __enter__(self):
        br.set_schedule(self.name)

    def __exit__(self, *exc):
        br.set_schedule("auto")


@pytest.mark.parametrize("seed", range(3))
def test_schur_stage_values(seed):
    F, G = synth.pair_deg6(seed)
    with eval_kernel("schur"):
        ps, vals = br.debug_values(F, G)
    for k, p in enumerate(ps):
        for a in range(vals.shape[1]):
            assert int(vals[k, a]) == resultant_at_mod(F, G, a, p), (k, a)


def test_schur_fallback_on_vanishing_leading_coefficients():
    # lc_y f = x - 5 vanishes at the point 5: the first pivot is f_m(a), so
    # that point falls back; lc_y g = x - 3 vanishes at 3, which leaves every
    # leading principal minor of S non-zero there (the formal degree is kept
    # by the generators themselves)
    F = [[1, 2, 3], [4, 5, 6], [-5, 1]]
    G = [[2, 0, 1], [-3, 1]]
    want = br.resultant(F, G)
    i0, f0 = br.schur_stats()
    with schedule("schur"):
        res, status = br.resultant_batch([("res", F, G, "y")])
    i1, f1 = br.schur_stats()
    assert status == [0] and res[0] == want
    say("instances", i1 - i0, "fallbacks", f1 - f0)
    assert i1 - i0 > 0
    assert f1 - f0 == 1  # one prime, one point


def test_schur_generic_pairs_have_no_fallback():
    pairs = [synth.pair_deg20(s) for s in range(4)]
    i0, f0 = br.schur_stats()
    with schedule("schur"):
        res, status = br.resultant_batch([("res", F, G, "y") for F, G in pairs])
    i1, f1 = br.schur_stats()
    assert status == [0] * 4
    assert res[0] == load("deg20_res_0.txt")[1]
    assert i1 - i0 == 4 * 48 * 401
    assert f1 - f0 == 0


@pytest.mark.parametrize("group", ["deg20", "capacity", "curve40"])
def test_schur_full_size_against_oracle_nodes(group):
    names = nodecheck.names(group)
    if group == "deg20":
        names = names[:3]
    jobs, recs = [], []
    for name in names:
        rec = nodecheck.case(group, name)
        kind, F, G, _ = nodecheck.inputs(rec)
        jobs.append((kind, F, G, "y"))
        recs.append(rec)
    say(group, len(jobs), "jobs")
    with schedule("schur"):
        res, status = br.resultant_batch(jobs)
    assert status == [0] * len(jobs)
    for R, rec in zip(res, recs):
        say("  ", rec["name"])
        nodecheck.check(R, rec)


def test_schur_two_rows_per_lane_at_the_top_of_the_range():
    rng = random.Random(3)
    F, _ = synth.random_rect(41, 60, 2, 0, 0, 24)
    G, _ = synth.random_rect(42, 60, 1, 0, 0, 24)
    want = br.resultant(F, G)            # Euclid (LDS kernel: m, n >= 32)
    with schedule("schur"):
        res, status = br.resultant_batch([("res", F, G, "y")])
    assert status == [0] and res[0] == want
    q = (1 << 61) - 1
    for a in [0, 1, rng.randint(2, 10**6)]:
        assert zx.evaluate(want, a) % q == resultant_at_mod(F, G, a, q)


def test_schur_mixed_batch_with_ineligible_jobs():
    jobs = [("res",) + synth.pair_deg6(1) + ("y",),
            ("res", [[1, 2, 3]], [[4, 5], [6, 7], [8, 9]], "y"),      # m = 0: Euclid's kernel
            ("disc", synth.curve_deg40(2, tdeg=12, bits=10), None, "y")]
    F, _ = synth.random_rect(43, 70, 1, 0, 0, 8)
    G, _ = synth.random_rect(44, 65, 1, 0, 0, 8)
    jobs.append(("res", F, G, "y"))                                    # r = 135 > 128
    with schedule("staged"):
        want, st0 = br.resultant_batch(jobs)
    with schedule("schur"):
        got, st1 = br.resultant_batch(jobs)
    assert st0 == st1 == [0] * len(jobs)
    assert got == want


def test_autotune_three_schedules():
    import torch
    pairs = [synth.pair_deg20(s) for s in range(32)]
    b = br.DeviceBatch([("res", F, G, "y") for F, G in pairs])
    chosen = b.autotune(reps=1)
    say("autotuner chose", chosen)
    assert chosen in ("staged", "fused", "schur")
    b.run()
    torch.cuda.synchronize()
    assert b.results()[0] == load("deg20_res_0.txt")[1]
