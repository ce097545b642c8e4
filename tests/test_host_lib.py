"""Host-side checks of the C-ABI library (no GPU): it loads, exports every
symbol include/bires.h declares, and its host-only planning is sound against
the oracle (degree bound, Hadamard coefficient bound, prime table)."""

import os
import re

import math

import pytest
import sympy as sp

import paper_1201_1548_amd as br
from oracle import zx
from oracle.resultant import discriminant_y, resultant_x, resultant_y
from paper_1201_1548_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bires.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bires_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = br.lib()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n


def test_prime_table():
    ps = br.primes(300)
    ceil = (2**32 - 1) // 3                        # 3p < 2^32: three-product reductions
    assert not any(sp.isprime(c) for c in range(ps[0] + 1, ceil + 1))
    assert all(2**30 < p and 3 * p < 2**32 for p in ps)
    assert all(a > b for a, b in zip(ps, ps[1:]))
    assert all(sp.isprime(p) for p in ps)
    # no prime skipped between consecutive table entries
    for a, b in zip(ps[:20], ps[1:21]):
        assert not any(sp.isprime(c) for c in range(b + 1, a))


def test_limb_marshalling_round_trip():
    vals = [0, 1, -1, 2**31 - 1, -2**31, 2**95 + 12345, -(2**200) + 7]
    L = br.limbs_needed(vals)
    assert br.limbs_to_ints(br.ints_to_limbs(vals, L)) == vals
    assert br.limbs_needed([2**31 - 1, -2**31]) == 1
    assert br.limbs_needed([2**31]) == 2


def _check_plan(F, G, R, kind="res", var="y"):
    D, P, log2B = br.plan(F, G, kind, var)
    assert zx.deg(R) <= D - 1
    if R:
        assert max(abs(c) for c in R).bit_length() <= log2B + 1
    ps = br.primes(P)
    M = 1
    for p in ps:
        M *= p
    assert math.log2(M) > log2B + 1.001              # M > 2^1.001 B (margin of the explicit CRT)
    deg, L = br.bounds(F, G, kind, var)
    assert deg >= D - 1
    assert L >= (max((abs(c) for c in R), default=0).bit_length() + 1 + 31) // 32
    return D, P


@pytest.mark.parametrize("inst", range(3))
def test_plan_bounds_deg6(inst):
    F, G = synth.pair_deg6(inst)
    D, P = _check_plan(F, G, resultant_y(F, G))
    assert D == 37


@pytest.mark.parametrize("seed", range(6))
def test_plan_bounds_random_shapes(seed):
    F, G = synth.random_rect(seed, 1 + seed % 4, 2 + seed % 3, 2 + (seed * 7) % 3, 1 + seed % 2, 20 + 9 * seed)
    _check_plan(F, G, resultant_y(F, G))
    _check_plan(F, G, resultant_x(F, G), var="x")
    _check_plan(F, None, discriminant_y(F), kind="disc")


def test_plan_deg20_prime_count():
    F, G = synth.pair_deg20(0)
    D, P, log2B = br.plan(F, G)
    assert D == 401
    assert 40 <= P <= 60


def test_bounds_reject_bad_arguments():
    with pytest.raises(br.BiresError):
        br.bounds([[1, 2]], None, kind="disc")     # y-degree 0 has no y-derivative resultant
