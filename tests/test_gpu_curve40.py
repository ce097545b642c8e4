"""Curve analysis: R = res(f, f_y; y) for dense total-degree-40
curves with 16-bit coefficients, and gcd(R, R') in Z[x].

At full size the oracle cannot form R by Bareiss in test time, so R is checked
on sampled outputs the oracle computes one by one: R(a) mod q for a 61-bit
prime q (determinant of the specialised Sylvester matrix over F_q, keeping the
formal degrees).  The gcd is checked by its defining properties: it divides R
and R' exactly, its cofactors are coprime (their gcd modulo a prime that does
not divide their leading coefficients is 1), its content is the gcd of the
contents of R and R', and its leading coefficient is positive.  A smaller
curve of the same construction is compared with the oracle in full.  (The
curve discriminants also have full-size parity through the oracle's node
digests in tests/test_gpu_fullsize.py.)"""

import math
import random

import pytest

import paper_1201_1548_amd as br
from oracle import zx
from oracle.gcd import gcd_mod_p, gcd_zx
from oracle.resultant import bi_diff_y, discriminant_y, resultant_at_mod
from paper_1201_1548_amd import synth

pytestmark = pytest.mark.gpu
Q = (1 << 61) - 1   # Mersenne prime, not in the prime table


def say(*a):
    print(*a, flush=True)


def check_R_samples(F, R, points):
    Fy = bi_diff_y(F)
    for a in points:
        assert zx.evaluate(R, a) % Q == resultant_at_mod(F, Fy, a, Q), a


def check_gcd(R, h):
    # h is the normalised gcd of R and R' exactly when it divides both, the
    # cofactors are coprime, its content is gcd(cont R, cont R') (the content
    # of a gcd is the gcd of the contents) and its leading coefficient is
    # positive; coprimality of the cofactors is checked modulo a large prime
    # that keeps their degrees (a common factor over Z stays common mod p)
    dR = zx.derivative(R)
    qa = zx.exact_div(R, h)
    qb = zx.exact_div(dR, h)
    assert h[-1] > 0
    assert zx.content(h) == math.gcd(zx.content(R), zx.content(dR))
    p = 2305843009213693951  # 2^61 - 1
    assert qa[-1] % p and qb[-1] % p
    assert gcd_mod_p(qa, qb, p) == [1]


def test_small_curve_full_oracle():
    F = synth.curve_deg40(7, tdeg=7, bits=16)
    say("small curve shaped like the degree-40 ones")
    R = br.discriminant(F)
    assert R == discriminant_y(F)
    dR = zx.derivative(R)
    assert br.gcd(R, dR) == gcd_zx(R, dR)


def test_curve_deg40_dense():
    F = synth.curve_deg40(0)
    say("dense total degree 40: discriminant")
    R = br.discriminant(F)
    assert len(R) - 1 <= 40 * 39
    rng = random.Random(3)
    check_R_samples(F, R, [0, 1, -2] + [rng.randint(-10**6, 10**6) for _ in range(3)])
    say("dense total degree 40: gcd(R, R')")
    h = br.gcd(R, zx.derivative(R))
    say("deg gcd =", len(h) - 1)
    check_gcd(R, h)


@pytest.mark.parametrize("square_k", [False, True])
def test_curve_deg40_singular_variants(square_k):
    F = synth.singular_curve_deg40(0, square_k=square_k, dk=20 if not square_k else 10)
    say("g^2 + h k%s" % ("^2" if square_k else ""), "ydeg", len(F) - 1)
    R = br.discriminant(F)
    rng = random.Random(4)
    check_R_samples(F, R, [0, 1] + [rng.randint(-10**5, 10**5) for _ in range(2)])
    h = br.gcd(R, zx.derivative(R))
    say("deg gcd =", len(h) - 1)
    check_gcd(R, h)
    if square_k:
        assert len(h) - 1 >= 1    # singular where g = k = 0: R has repeated roots
