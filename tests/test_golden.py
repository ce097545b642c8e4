"""The stored expected values under tests/golden/ are the oracle's and still match the inputs.

Every golden file records the digest of the synthetic inputs it was computed
from; a changed generator fails here.  Each stored resultant is also checked
against the evaluation homomorphism R(a) = det S(f(a, y), g(a, y)) at a few
integer points (independent of the Z[x] determinant that produced it) and
against the Bezout-type degree bound of Section 2.
"""

import os

import pytest

from oracle import zx
from oracle.resultant import resultant_at, resultant_y
from paper_1201_1548_amd import synth
from tests.golden.make_golden import input_digest, load

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("inst", range(4))
def test_deg6_golden(inst):
    F, G = synth.pair_deg6(inst)
    digest, R = load("deg6_res_%d.txt" % inst)
    assert digest == input_digest(F, G)
    assert R == resultant_y(F, G)
    for a in (-2, 0, 5):
        assert zx.evaluate(R, a) == resultant_at(F, G, a)


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "deg20_res_0.txt")),
                    reason="degree-20 golden file not generated")
def test_deg20_golden_spot_values():
    F, G = synth.pair_deg20(0)
    digest, R = load("deg20_res_0.txt")
    assert digest == input_digest(F, G)
    assert len(R) - 1 <= 400
    for a in (0, 1, -1, 3):
        assert zx.evaluate(R, a) == resultant_at(F, G, a)


# ---------------------------------------------------------------------------
# node-value digests (tests/golden/nodes_*.json) and the check built on them

import math  # noqa: E402

import sympy  # noqa: E402

from oracle.bounds import coeff_bound, degree_bound  # noqa: E402
from oracle.resultant import resultant_at_mod  # noqa: E402
from tests import nodecheck  # noqa: E402
from tests.golden.make_node_digests import GROUPS, load_group, node_digest, operands, primes_for  # noqa: E402


@pytest.mark.parametrize("group", GROUPS)
def test_node_digest_files_are_the_oracles(group):
    doc = load_group(group)
    assert doc["cases"]
    for rec in doc["cases"]:
        kind, F, G, G2 = nodecheck.inputs(rec)
        assert input_digest(F, G) == rec["inputs_sha256"], rec["name"]
        A, B = operands(kind, F, G2)
        assert degree_bound(A, B) + 1 == rec["D"]
        primes = [int(q) for q in rec["primes"]]
        assert len(set(primes)) == len(primes) == len(rec["digests"])
        assert all(sympy.isprime(q) for q in primes)
        assert math.prod(primes) > 2 * coeff_bound(A, B)
        # one stored value recomputed by the oracle here
        a, v = rec["samples_prime0"][0]
        assert resultant_at_mod(A, B, a, primes[0]) == int(v), rec["name"]


def _digest_record(F, G, R_true):
    D = degree_bound(F, G) + 1
    ps = primes_for(coeff_bound(F, G))
    vals = [[resultant_at_mod(F, G, a, q) for a in range(D)] for q in ps]
    return {"D": D, "primes": [str(q) for q in ps], "digests": [node_digest(v) for v in vals],
            "samples_prime0": [[0, str(vals[0][0])]], "Q": math.prod(ps)}


def test_node_check_accepts_the_oracle_and_rejects_planted_mistakes(monkeypatch):
    F, G = synth.pair_deg6(0)
    _, R = load("deg6_res_0.txt")
    rec = _digest_record(F, G, R)
    rec.update({"gen": "pair_deg6", "args": [0], "kind": "res", "inputs_sha256": input_digest(F, G),
                "name": "deg6_0"})
    nodecheck.check(R, rec)
    wrong = list(R)
    wrong[7] += 1                                   # one coefficient off by one
    with pytest.raises(AssertionError):
        nodecheck.check(wrong, rec)
    shifted = list(R)
    shifted[3] += rec["Q"]                          # same residues, outside the range
    with pytest.raises(AssertionError):
        nodecheck.check(shifted, rec)
    with pytest.raises(AssertionError):             # degree above the bound
        nodecheck.check(R + [1], rec)
    with pytest.raises(AssertionError):             # wrong sign
        nodecheck.check([-c for c in R], rec)
    with pytest.raises(AssertionError):             # coefficients in reversed order
        nodecheck.check(R[::-1], rec)


def test_degree_and_coefficient_bounds_hold_and_are_attained():
    # bounds of the Sylvester matrix (Leibniz expansion) against the oracle's R
    import random
    rng = random.Random(11)
    for seed in range(12):
        a, b, c, d = (rng.randint(0, 4) for _ in range(4))
        F, G = synth.random_rect(5000 + seed, a, b, c, d, rng.randint(2, 30), zero_frac=0.3 * (seed % 2))
        R = resultant_y(F, G)
        if R:
            assert len(R) - 1 <= degree_bound(F, G)
            assert max(abs(v) for v in R) <= coeff_bound(F, G)
    # generic dense pairs attain the degree bound n t_f + m t_g - m n
    for inst in range(4):
        F, G = synth.pair_deg6(inst)
        assert degree_bound(F, G) == len(load("deg6_res_%d.txt" % inst)[1]) - 1 == 36
    # f = 2x (y-free), g of y-degree 3: R = f^3 = 8 x^3 attains the coefficient bound
    F, G = [[0, 2]], [[1], [0], [0], [1]]
    assert resultant_y(F, G) == [0, 0, 0, 8] and coeff_bound(F, G) == 8 and degree_bound(F, G) == 3
    # every permutation meets a zero entry: bound -1 (det = 0)
    assert degree_bound([[0], [0], [1]], [[0], [0], [1]]) == -1
