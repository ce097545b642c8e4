"""Pins of the Z[x] helpers and of the gcd oracle against independent facts.

* Kronecker multiplication against the schoolbook convolution (definition);
* exact division: round trip, and refusal of an inexact division;
* gcd_zx against sympy's gcd over Z[x] (library routine) and against the
  defining properties: it divides both inputs in Z[x], the cofactors are coprime
  over Q (sympy), and gcd(A C, B C) = C gcd(A, B) for a planted common factor;
* gcd over F_p against sympy's gcd over GF(p).
"""

import random

import pytest
import sympy as sp

from oracle import zx
from oracle.gcd import gcd_mod_p, gcd_q_euclid, gcd_zx, prem

X = sp.symbols("x")


def rpoly(rng, d, lo=-20, hi=20):
    a = [rng.randint(lo, hi) for _ in range(d + 1)]
    a[-1] = a[-1] or 1
    return a


def schoolbook(a, b):
    if not a or not b:
        return []
    out = [0] * (len(a) + len(b) - 1)
    for i, u in enumerate(a):
        for j, v in enumerate(b):
            out[i + j] += u * v
    return zx.trim(out)


def to_sp(a):
    return sp.Poly(list(reversed(a)) or [0], X)


def from_sp(P):
    return zx.trim([int(c) for c in reversed(P.all_coeffs())]) if not P.is_zero else []


@pytest.mark.parametrize("seed", range(10))
def test_kronecker_mul_matches_schoolbook(seed):
    rng = random.Random(seed)
    a = rpoly(rng, rng.randint(0, 30), -(1 << 70), 1 << 70)
    b = rpoly(rng, rng.randint(0, 30), -(1 << 40), 1 << 40)
    assert zx.mul(a, b) == schoolbook(a, b)


@pytest.mark.parametrize("seed", range(10))
def test_exact_div_round_trip(seed):
    rng = random.Random(100 + seed)
    q = rpoly(rng, rng.randint(0, 25), -(1 << 50), 1 << 50)
    d = rpoly(rng, rng.randint(1, 25), -(1 << 30), 1 << 30)
    assert zx.exact_div(zx.mul(q, d), d) == q
    with pytest.raises(ArithmeticError):
        zx.exact_div(zx.add(zx.mul(q, d), [1]), d)


@pytest.mark.parametrize("seed", range(10))
def test_gcd_matches_sympy_with_planted_factor(seed):
    rng = random.Random(200 + seed)
    C = rpoly(rng, rng.randint(0, 4), -9, 9)
    A = rpoly(rng, rng.randint(0, 5), -9, 9)
    B = rpoly(rng, rng.randint(0, 5), -9, 9)
    a, b = zx.mul(A, C), zx.mul(B, C)
    h = gcd_zx(a, b)
    assert h == from_sp(sp.gcd(to_sp(a), to_sp(b)))
    # defining properties
    qa, qb = zx.exact_div(a, h), zx.exact_div(b, h)
    assert sp.gcd(to_sp(qa), to_sp(qb)).degree() == 0
    assert h[-1] > 0
    # planted factor: gcd(A C, B C) = C gcd(A, B) up to the sign convention
    cg = zx.mul(C, gcd_zx(A, B))
    assert h == (cg if cg[-1] > 0 else zx.neg(cg))


def test_gcd_normalisation_edges():
    assert gcd_zx([], []) == []
    assert gcd_zx([0, -2, -4], []) == [0, 2, 4]
    assert gcd_zx([], [6]) == [6]
    assert gcd_zx([6, 4], [9, 6]) == [3, 2]        # content gcd times primitive gcd
    assert gcd_zx([4], [6]) == [2]


@pytest.mark.parametrize("seed", range(6))
def test_gcd_mod_p_matches_sympy(seed):
    rng = random.Random(300 + seed)
    p = 1000003
    C = rpoly(rng, rng.randint(1, 4), 0, p - 1)
    a = zx.mul(rpoly(rng, 4, 0, p - 1), C)
    b = zx.mul(rpoly(rng, 3, 0, p - 1), C)
    ref = sp.Poly(list(reversed(a)), X, modulus=p).gcd(sp.Poly(list(reversed(b)), X, modulus=p))
    ref = [int(c) % p for c in reversed(ref.all_coeffs())]
    assert gcd_mod_p(a, b, p) == ref


@pytest.mark.parametrize("seed", range(6))
def test_primitive_prs_equals_rational_euclid(seed):
    rng = random.Random(400 + seed)
    C = rpoly(rng, rng.randint(0, 3), -9, 9)
    a = zx.mul(rpoly(rng, rng.randint(0, 6), -30, 30), C)
    b = zx.mul(rpoly(rng, rng.randint(0, 6), -30, 30), C)
    assert gcd_zx(a, b) == gcd_q_euclid(a, b)


def test_pseudo_remainder_definition():
    rng = random.Random(7)
    u, v = rpoly(rng, 7, -50, 50), rpoly(rng, 3, -50, 50)
    r = prem(u, v)
    # lc(v)^(deg u - deg v + 1) u = q v + r with deg r < deg v, checked over Q
    q, rq = zx.divmod_q([c * v[-1] ** 5 for c in u], v)
    assert [int(x) for x in rq] == r and all(x.denominator == 1 for x in q)
