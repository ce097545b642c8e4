"""bench.py's local helpers: the Kronecker product it uses to check square-free
decompositions, and its reader of the stored oracle output."""
import os
import random

import bench
from tests.golden.make_golden import load


def _schoolbook(a, b):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    while out and out[-1] == 0:
        out.pop()
    return out


def test_kronecker_product_matches_schoolbook():
    rng = random.Random(3)
    for _ in range(200):
        a = [rng.randint(-(1 << rng.randint(1, 300)), 1 << 200) for _ in range(rng.randint(1, 12))]
        b = [rng.randint(-(1 << 90), 1 << rng.randint(1, 300)) for _ in range(rng.randint(1, 12))]
        a[-1] = a[-1] or 1
        b[-1] = b[-1] or -1
        assert bench._zx_mul(a, b) == _schoolbook(a, b)
    assert bench._zx_mul([], [1, 2]) == []
    assert bench._zx_derivative([5, 3, 0, 4]) == [3, 0, 12]
    assert bench._zx_derivative([7]) == []


def test_golden_reader_matches_the_loader():
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    for name in ("deg6_res_0.txt", "deg20_res_0.txt"):
        assert bench.read_golden(os.path.join(here, name)) == load(name)[1]
