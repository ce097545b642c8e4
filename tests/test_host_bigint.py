"""The host big-integer helpers of the gcd (Knuth-D division, gcd, products,
two's-complement conversion) against Python's integers, through a small
native driver built with g++ (no GPU)."""

import math
import os
import random
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("bigint") / "bigint_driver")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "native", "bigint_driver.cpp"),
                    os.path.join(ROOT, "paper_1201_1548_amd", "csrc", "bigint.cpp")], check=True)
    return exe


def hx(v):
    return ("-" if v < 0 else "") + format(abs(v), "x")


def run(exe, lines):
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    return out.stdout.split("\n")


def rnd(rng, maxbits):
    b = rng.randint(1, maxbits)
    v = rng.getrandbits(b)
    if rng.random() < 0.3:   # long runs of ones and zeros stress the qhat correction
        v |= ((1 << rng.randint(1, b)) - 1)
    return v


def test_divmod_mul_gcd(driver):
    rng = random.Random(1)
    cases = []
    for _ in range(400):
        a, b = rnd(rng, 3000), rnd(rng, 1500) or 1
        cases.append((a, b))
    lines = ["divmod %s %s" % (hx(a), hx(b)) for a, b in cases]
    lines += ["mul %s %s" % (hx(a), hx(-b)) for a, b in cases]
    lines += ["gcd %s %s" % (hx(a * 7919), hx(b * 7919)) for a, b in cases]
    out = run(driver, lines)
    n = len(cases)
    for i, (a, b) in enumerate(cases):
        q, r = out[i].split()
        assert int(q, 16) == a // b and int(r, 16) == a % b, (a, b)
        assert int(out[n + i].replace("-", ""), 16) == a * b and (out[n + i].startswith("-") or a * b == 0)
        assert int(out[2 * n + i], 16) == math.gcd(a * 7919, b * 7919)


def test_twos_modsmall_divexact(driver):
    rng = random.Random(2)
    lines, exp = [], []
    for _ in range(200):
        v = rnd(rng, 500) * rng.choice([1, -1])
        L = (v.bit_length() + 1 + 31) // 32 + rng.randint(0, 2)
        lines.append("twos %s %x" % (hx(v), L))
        exp.append(("twos", v))
        p = rng.choice([2147483647, 2147483629, 1073741827])
        lines.append("modsmall %s %x" % (hx(v), p))
        exp.append(("mod", v % p))
        d = rnd(rng, 300) or 3
        lines.append("divexact %s %s" % (hx(v * d), hx(-d)))
        exp.append(("dx", -v))
        lines.append("divexact %s %s" % (hx(v * d + 1), hx(d)))
        exp.append(("dx", None if d > 1 else v * d + 1))
    out = run(driver, lines)
    for line, (kind, val) in zip(out, exp):
        if kind == "twos":
            s, bits = line.split()
            assert int(s, 16) == val and int(bits) == abs(val).bit_length()
        elif kind == "mod":
            assert int(line, 16) == val
        else:
            assert (line == "inexact") if val is None else int(line, 16) == val
