"""Square-free decomposition by Yun's algorithm on the device gcd with exact
cofactors (bires_squarefree) against the oracle's decomposition
(oracle/squarefree.py): planted factorisations with known multiplicities, the
discriminant of a singular curve, and edge cases.  Decompositions are unique
under the normalisation (signed content, primitive factors with positive
leading coefficient), so the comparison is exact."""
import random

import pytest

import paper_1201_1548_amd as br
from oracle import zx
from oracle.gcd import gcd_zx
from oracle.squarefree import derivative, expand, squarefree_yun
from paper_1201_1548_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def _random_factor(rng, deg, bits):
    while True:
        a = [rng.randint(-(1 << bits), 1 << bits) for _ in range(deg)] + [rng.randint(1, 1 << bits)]
        a = zx.primitive_part(a)
        if len(a) == deg + 1 and gcd_zx(a, derivative(a)) == [1]:
            return a


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_planted_decompositions_match_the_oracle(seed):
    rng = random.Random(300 + seed)
    r = [rng.choice([1, -1, 12, -7 * 2 ** 40])]
    planted = []
    for mult in range(1, 5):
        if rng.random() < 0.25 and mult < 4:
            continue  # a missing multiplicity: a_mult = 1
        a = _random_factor(rng, rng.randint(1, 12), rng.choice([40, 90, 200]))
        planted.append((mult, a))
        for _ in range(mult):
            r = zx.mul(r, a)
    say("planted", seed, "deg", len(r) - 1, [(m, len(a) - 1) for m, a in planted])
    got = br.squarefree(r)
    want = squarefree_yun(r)
    assert got == want
    assert expand(*got) == zx.trim(r)


def test_discriminant_of_a_singular_curve():
    # f = g^2 + h k^2: res(f, f_y; y) has repeated factors
    F = synth.singular_curve_deg40(0, dg=4, dh=4, dk=3, bits=6, square_k=True)
    R = br.discriminant(F)
    say("singular curve discriminant deg", len(R) - 1)
    u, fs = br.squarefree(R)
    assert (u, fs) == squarefree_yun(R)
    assert expand(u, fs) == R
    assert len(fs) >= 2


def test_edge_cases():
    say("squarefree edge cases")
    assert br.squarefree([]) == (0, [])
    assert br.squarefree([-9]) == (-9, [])
    assert br.squarefree([0, 5]) == (5, [[0, 1]])
    assert br.squarefree([0, 0, -1, 1]) == (1, [[-1, 1], [0, 1]])
    a = [3, -1, 0, 2]
    r5 = [1]
    for _ in range(5):
        r5 = zx.mul(r5, a)
    assert br.squarefree(zx.scale(r5, -3)) == squarefree_yun(zx.scale(r5, -3)) == (-3, [[1], [1], [1], [1], a])
