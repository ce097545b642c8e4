"""Parity of the modular gcd (HIP path through the C ABI) with the oracle's gcd
in Z[x] (Euclid over Q, then content), bit-exact."""

import random

import pytest

import paper_1201_1548_amd as br
from oracle import zx
from oracle.gcd import gcd_mod_p, gcd_zx
from oracle.resultant import bi_mul, discriminant_y
from paper_1201_1548_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rpoly(rng, d, bits):
    a = [rng.randint(-(1 << bits), 1 << bits) for _ in range(d + 1)]
    a[-1] = a[-1] or 1
    return a


@pytest.mark.parametrize("seed", range(8))
def test_planted_common_factor(seed):
    rng = random.Random(seed)
    C = rpoly(rng, rng.randint(0, 6), rng.choice([4, 30, 90]))
    A = rpoly(rng, rng.randint(1, 40), rng.choice([8, 40, 120]))
    B = rpoly(rng, rng.randint(1, 40), rng.choice([8, 40, 120]))
    a, b = zx.mul(A, C), zx.mul(B, C)
    say("planted factor seed", seed, len(a), len(b))
    assert br.gcd(a, b) == gcd_zx(a, b)


def test_contents_and_signs():
    rng = random.Random(11)
    C = rpoly(rng, 3, 10)
    a = zx.scale(zx.mul(rpoly(rng, 5, 10), C), -12)
    b = zx.scale(zx.mul(rpoly(rng, 4, 10), C), 18)
    say("contents and signs")
    assert br.gcd(a, b) == gcd_zx(a, b)
    assert br.gcd([6, 4], [9, 6]) == [3, 2]
    assert br.gcd([4], [6]) == [2]
    assert br.gcd([0, -2, -4], []) == [0, 2, 4]
    assert br.gcd([], []) == []
    assert br.gcd([5, 0, 3], [7]) == [1]


def test_coprime_large():
    # certificate instead of the oracle: gcd modulo a 61-bit prime not dividing
    # the leading coefficients is 1, so a and b are coprime over Q
    rng = random.Random(12)
    a, b = rpoly(rng, 200, 60), rpoly(rng, 150, 60)
    say("coprime large")
    q = (1 << 61) - 1
    assert a[-1] % q and b[-1] % q and gcd_mod_p(a, b, q) == [1]
    import math
    c = math.gcd(zx.content(a), zx.content(b))
    assert br.gcd(a, b) == [c]


def test_high_power_common_factor():
    rng = random.Random(13)
    C = rpoly(rng, 2, 5)
    a = zx.mul(zx.power(C, 7), rpoly(rng, 3, 5))
    b = zx.mul(zx.power(C, 5), rpoly(rng, 6, 5))
    say("high power")
    assert br.gcd(a, b) == gcd_zx(a, b)


def test_discriminant_gcd_with_derivative():
    # f = g^2 + h k^2 is singular where g = k = 0, so R = res(f, f_y; y) has repeated roots
    f = synth.singular_curve_deg40(0, dg=3, dh=2, dk=2, bits=4, square_k=True)
    say("gcd(R, R') of a singular curve")
    R = br.discriminant(f)
    assert R == discriminant_y(f)
    dR = zx.derivative(R)
    h = br.gcd(R, dR)
    assert h == gcd_zx(R, dR)
    assert len(h) - 1 >= 1


def test_device_memory_gcd():
    import torch
    import numpy as np
    rng = random.Random(14)
    C = rpoly(rng, 4, 20)
    a, b = zx.mul(rpoly(rng, 9, 20), C), zx.mul(rpoly(rng, 7, 20), C)
    La = br.limbs_needed(a)
    Lb = br.limbs_needed(b)
    ta = torch.from_numpy(br.ints_to_limbs(a, La).view(np.int32)).cuda()
    tb = torch.from_numpy(br.ints_to_limbs(b, Lb).view(np.int32)).cuda()
    ua = br.Upoly(len(a) - 1, La, ta.data_ptr())
    ub = br.Upoly(len(b) - 1, Lb, tb.data_ptr())
    import ctypes
    deg = ctypes.c_int32()
    L = ctypes.c_int32()
    assert br.lib().bires_gcd_bounds(ctypes.byref(ua), ctypes.byref(ub), ctypes.byref(deg), ctypes.byref(L)) == 0
    out = torch.zeros((deg.value + 1, L.value), dtype=torch.int32, device="cuda")
    uo = br.Upoly(deg.value, L.value, out.data_ptr())
    code = br.lib().bires_gcd(ctypes.byref(ua), ctypes.byref(ub), ctypes.byref(uo), br.MEM_DEVICE,
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert code == 0
    got = br.limbs_to_ints(out[: uo.degree + 1].cpu().numpy().view(np.uint32))
    assert got == gcd_zx(a, b)
