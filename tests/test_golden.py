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
