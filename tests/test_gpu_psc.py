"""Principal subresultant coefficients modulo one prime and the N^- / N^+
test (Section 3.2.2) against the oracle (oracle.subresultants).

* psc's: every coefficient of every sr_i mod p equals the oracle's
  (determinant definition over Z[x], reduced mod p) on pairs of every shape:
  m > n, m < n, m = n, the three kinds, leading coefficients that vanish at
  some points, at every point or modulo p (formal degrees kept), defective
  remainder sequences (common factors), multi-limb coefficients, var = x;
* at the degree-40 curve's size (D = 1561), sampled (point, index) values
  against the oracle's determinants over F_p of the specialised matrices;
* N^- and N^+ equal the oracle's on small singular and non-singular curves
  for two primes, and at the degree-40 size satisfy N^- <= N^+, with
  N^- = N^+ = deg R* (n_y - 1) for the generic dense curve (only simple
  tangencies: one double root per x-critical fiber).
"""

import random

import pytest

import paper_1201_1548_amd as br
from oracle import zx
from oracle.resultant import bi_add, bi_diff_y, bi_mul, bi_transpose, bi_trim, discriminant_y, resultant_y
from oracle.squarefree import squarefree_yun
from oracle.subresultants import (bi_diff_x, fp, lower_bound, polar_resultant_y, psc_at_mod, psc_zx,
                                  upper_bound)
from paper_1201_1548_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rand_bi(rng, ydeg, xdeg, bits):
    h = 1 << (bits - 1)
    F = [[rng.randint(-h, h - 1) for _ in range(xdeg + 1)] for _ in range(ydeg + 1)]
    if not any(F[-1]):
        F[-1][0] = 1
    return F


def want_psc(F, G, p):
    return [fp(s, p) for s in psc_zx(F, G)]


def primes2():
    ps = br.primes(40)
    return [ps[0], ps[37]]


@pytest.mark.parametrize("seed", range(8))
def test_psc_random_shapes(seed):
    rng = random.Random(seed)
    m, n = rng.randint(1, 6), rng.randint(1, 6)
    bits = rng.choice([6, 20, 40, 90])
    F, G = rand_bi(rng, m, rng.randint(0, 4), bits), rand_bi(rng, n, rng.randint(0, 4), bits)
    say("seed", seed, "m", m, "n", n, "bits", bits)
    for p in primes2():
        q, rows = br.psc(F, G, prime=p)
        assert q == p
        assert rows == want_psc(F, G, p)


def test_psc_kinds_and_var_x():
    rng = random.Random(50)
    F = rand_bi(rng, 5, 4, 24)
    p = primes2()[1]
    assert br.psc(F, kind="disc", prime=p)[1] == want_psc(F, bi_diff_y(F), p)
    assert br.psc(F, kind="polar", prime=p)[1] == want_psc(bi_diff_x(F), bi_diff_y(F), p)
    G = rand_bi(rng, 3, 5, 24)
    assert br.psc(F, G, var="x", prime=p)[1] == want_psc(bi_transpose(F), bi_transpose(G), p)


def test_psc_formal_degrees():
    p = primes2()[0]
    # lc_y f = x - 3 vanishes at the point 3; lc_y g = x - 3 as well at the same point
    F = [[1, 2, 0], [3, -1, 4], [-3, 1]]
    G = [[5, 0, 1], [-3, 1]]
    assert br.psc(F, G, prime=p)[1] == want_psc(F, G, p)
    # leading rows vanishing at several points, m < n and m = n
    F2 = [[2, 1], [1, 1, 1], [0, -2, 1]]          # lc = x^2 - 2x: zero at 0 and 2
    G2 = [[1], [0, 1], [4, 0, -1], [-6, 1, 1]]    # lc = x^2 + x - 6: zero at 2
    assert br.psc(F2, G2, prime=p)[1] == want_psc(F2, G2, p)
    assert br.psc(G2, F2, prime=p)[1] == want_psc(G2, F2, p)
    G3 = [[1, 5], [0, 1], [0, 1, -1]]             # m = n = 2, lc zero at 0 in both
    assert br.psc(F2, G3, prime=p)[1] == want_psc(F2, G3, p)
    # leading coefficient divisible by p: the formal degree is kept
    F4 = [[1, 2], [3, 4], [p, 2 * p]]
    G4 = [[7, 1], [1, -1]]
    assert br.psc(F4, G4, prime=p)[1] == want_psc(F4, G4, p)


def test_psc_defective_sequences():
    p = primes2()[1]
    lin = [[0, -1], [1]]                   # y - x
    rng = random.Random(7)
    A, B = rand_bi(rng, 3, 2, 12), rand_bi(rng, 2, 2, 12)
    F, G = bi_mul(lin, A), bi_mul(lin, B)  # common factor: sr_0 = 0
    rows = br.psc(F, G, prime=p)[1]
    assert rows == want_psc(F, G, p)
    assert rows[0] == []
    sq = bi_mul(lin, lin)
    F2, G2 = bi_mul(sq, A), bi_mul(sq, B)  # two common roots: sr_0 = sr_1 = 0
    rows = br.psc(F2, G2, prime=p)[1]
    assert rows == want_psc(F2, G2, p)
    assert rows[0] == [] and rows[1] == []
    # degree gaps in the remainder sequence: sparse y-structure
    F3 = [[1, 1], [], [], [0, 2], [], [3]]
    G3 = [[2], [], [1, 0, 1]]
    assert br.psc(F3, G3, prime=p)[1] == want_psc(F3, G3, p)


def test_psc_multilimb_and_constant_operand():
    rng = random.Random(9)
    p = primes2()[0]
    F, G = rand_bi(rng, 4, 3, 200), rand_bi(rng, 3, 3, 150)
    assert br.psc(F, G, prime=p)[1] == want_psc(F, G, p)
    # n = 0: sr_0 = g^m
    G0 = [[3, 0, 2]]
    assert br.psc(F, G0, prime=p)[1] == want_psc(F, G0, p)


def test_psc_rejects_other_primes_and_zero():
    F = [[1, 2], [3]]
    with pytest.raises(br.BiresError):
        br.psc(F, F, prime=1000003)
    with pytest.raises(br.BiresError):
        br.psc(F, [[0]], prime=br.primes(1)[0])


def test_psc_curve_deg40_sampled():
    F = synth.curve_deg40(0)
    p = primes2()[1]
    say("psc of (f, f_y), dense total degree 40")
    q, rows = br.psc(F, kind="disc", prime=p)
    assert len(rows) == 40
    Fy = bi_diff_y(F)
    rng = random.Random(1)
    for a in [0, 777] + [rng.randrange(p) for _ in range(1)]:
        want = psc_at_mod(F, Fy, a, p)
        got = [zx.evaluate(r, a) % p if r else 0 for r in rows]
        assert got == want, a


# ---------------------------------------------------------------- N^-, N^+

def rstar_of(R):
    u, fs = squarefree_yun(R)
    out = [1]
    for a in fs:
        out = zx.mul(out, a)
    return out


def small_curves():
    rng = random.Random(21)
    out = []
    for k in range(3):
        g = synth.dense_signed(synth.rng_for(7000 + k), 2, 4)
        h = synth.dense_signed(synth.rng_for(7100 + k), 2, 4)
        kk = synth.dense_signed(synth.rng_for(7200 + k), 1, 4)
        F = bi_add(bi_mul(g, g), bi_mul(h, bi_mul(kk, kk)))   # singular where g = k = 0
        out.append(bi_trim(F))
    out.append(bi_trim(synth.curve_deg40(3, tdeg=6, bits=8)))
    out.append(bi_trim([[0, 0, 0, -1], [], [1]]))             # cusp y^2 = x^3
    return [F for F in out if len(F[-1]) == 1]               # constant lc_y (no vertical asymptote)


@pytest.mark.parametrize("idx", range(5))
def test_fiber_bounds_small_curves(idx):
    curves = small_curves()
    if idx >= len(curves):
        pytest.skip("fewer curves with a constant leading coefficient")
    F = curves[idx]
    R = discriminant_y(F)
    Rs = rstar_of(R)
    Q = polar_resultant_y(F)
    say("curve", idx, "deg R", len(R) - 1, "deg R*", len(Rs) - 1)
    for p in primes2():
        nm, npl, flags = br.fiber_bounds(F, Rs, len(R) - 1, prime=p)
        assert flags == 0
        assert nm == lower_bound(F, Rs, p)
        assert npl == upper_bound(F, R, Rs, Q, p)
        assert nm <= npl


def test_fiber_bounds_curve_deg40():
    for name, F in (("dense", synth.curve_deg40(0)),
                    ("g2_hk2", synth.singular_curve_deg40(0, square_k=True, dk=10))):
        R = br.discriminant(F)
        u, fs = br.squarefree(R)
        Rs = [1]
        for a in fs:
            Rs = zx.mul(Rs, a)
        ny = len(bi_trim(F)) - 1
        nm, npl, flags = br.fiber_bounds(F, Rs, len(R) - 1)
        say(name, "deg R", len(R) - 1, "deg R*", len(Rs) - 1, "N-", nm, "N+", npl, "flags", flags)
        assert flags == 0
        assert nm <= npl
        if name == "dense" and len(Rs) == len(R):
            assert nm == npl == (len(Rs) - 1) * (ny - 1)
