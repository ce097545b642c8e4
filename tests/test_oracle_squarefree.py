"""Pins of the oracle's square-free decomposition (oracle/squarefree.py):
planted factorisations with known multiplicities, and the defining
properties (reconstruction, square-free and pairwise coprime factors)."""
import random

from oracle import zx
from oracle.gcd import gcd_zx
from oracle.squarefree import derivative, expand, squarefree_yun


def _prim_pos(a):
    a = zx.primitive_part(zx.trim(a))
    return [-c for c in a] if a[-1] < 0 else a


def _random_sqfree(rng, deg, bits, avoid=()):
    # random primitive polynomials are square-free and coprime to given ones
    # with overwhelming probability; the loop makes sure
    while True:
        a = [rng.randint(-(1 << bits), 1 << bits) for _ in range(deg)] + [rng.randint(1, 1 << bits)]
        a = _prim_pos(a)
        if len(a) != deg + 1:
            continue
        if gcd_zx(a, derivative(a)) != [1]:
            continue
        if all(gcd_zx(a, b) == [1] for b in avoid):
            return a


def test_planted_multiplicities():
    rng = random.Random(11)
    for trial in range(6):
        a1 = _random_sqfree(rng, rng.randint(1, 6), 20)
        a2 = _random_sqfree(rng, rng.randint(1, 5), 20, [a1])
        a3 = _random_sqfree(rng, rng.randint(1, 4), 20, [a1, a2])
        u = rng.choice([1, -1, 6, -35])
        r = zx.mul(zx.mul(zx.scale(a1, u), zx.mul(a2, a2)), zx.mul(a3, zx.mul(a3, a3)))
        assert squarefree_yun(r) == (u, [a1, a2, a3]), trial


def test_missing_multiplicity_and_pure_power():
    rng = random.Random(12)
    a1 = _random_sqfree(rng, 3, 16)
    a3 = _random_sqfree(rng, 2, 16, [a1])
    r = zx.mul(a1, zx.mul(a3, zx.mul(a3, a3)))
    assert squarefree_yun(r) == (1, [a1, [1], a3])
    a = _random_sqfree(rng, 4, 16)
    r5 = [1]
    for _ in range(5):
        r5 = zx.mul(r5, a)
    assert squarefree_yun(zx.scale(r5, -3)) == (-3, [[1], [1], [1], [1], a])


def test_squarefree_and_constant_inputs():
    rng = random.Random(13)
    a = _random_sqfree(rng, 7, 30)
    assert squarefree_yun(zx.scale(a, 4)) == (4, [a])
    assert squarefree_yun([0, 0]) == (0, [])
    assert squarefree_yun([-9]) == (-9, [])
    assert squarefree_yun([0, 5]) == (5, [[0, 1]])
    # x^2 (x - 1): multiplicities 1 and 2
    assert squarefree_yun([0, 0, -1, 1]) == (1, [[-1, 1], [0, 1]])


def test_reconstruction_and_defining_properties():
    rng = random.Random(14)
    for trial in range(8):
        parts = [_random_sqfree(rng, rng.randint(1, 4), 12) for _ in range(3)]
        r = [rng.randint(-5, 5) or 1]
        for i, a in enumerate(parts):
            for _ in range(rng.randint(1, 3)):
                r = zx.mul(r, a)
        u, fs = squarefree_yun(r)
        assert expand(u, fs) == zx.trim(r)
        assert fs and len(fs[-1]) >= 2
        for i, a in enumerate(fs):
            assert a[-1] > 0 and zx.content(a) == 1
            assert len(a) == 1 or gcd_zx(a, derivative(a)) == [1]
            for b in fs[i + 1:]:
                assert gcd_zx(a, b) == [1]
