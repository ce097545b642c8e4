"""CPU model of the evaluation/elimination arithmetic of the HIP kernel.

The univariate-resultant kernel computes, per (prime p, point a):

* f_j(a) in Montgomery form as an exact 96-bit sum S = sum_i c_i,M (a^i)_M,
  reduced by one REDC of (S mod 2^32) + (S >> 64) R^2 plus the middle word;
  rows longer than 24 coefficients in chunks of 24 combined by Horner's rule;
* the determinant of the Sylvester matrix (Section 2) over F_p by Euclid's
  algorithm without inverses: a - b + 1 eliminations per step (two of them
  fused into one pass when a = b + 1), formal-degree rules for vanishing
  leading coefficients, and the exponent of lc(B) split into prefix products.

This module restates that arithmetic in Python integers with the same word
bounds (asserted) and checks it against the oracle's determinant of the
Sylvester matrix mod p.  It pins the algebra of the kernel design; the GPU
parity tests pin the kernel itself.
"""

import random

import pytest

from oracle.resultant import det_mod, sylvester

R = 1 << 32
CEIL = (R - 1) // 3          # the table's primes lie in (2^30, 2^32 / 3)
PRIMES = [1431655751, 1431655747, 1431655739, 1073741827, 1073741831]


def redc(t, p):
    pinv = (-pow(p, -1, R)) % R
    assert 0 <= t < p * R
    m = (t % R) * pinv % R
    u = t + m * p
    assert u < 1 << 64
    r = u >> 32
    assert r < 2 * p
    return r - p if r >= p else r


def mont(x, p):
    return x * R % p


def mmul(a, b, p):
    return redc(a * b, p)


def mdot2(a, b, c, d, p):
    return redc(a * b + c * d, p)


def mdot3(a, b, c, d, e, f, p):
    return redc(a * b + c * d + e * f, p)


def mneg(x, p):
    return (p - x) % p


def reduce32(x, p):
    assert 0 <= x < R
    x = min(x, (x - 2 * p) % R)
    return min(x, (x - p) % R)


def fold96(S, p):
    lo_lo, lo_hi, hi = S & (R - 1), (S >> 32) & (R - 1), S >> 64
    assert hi < R - 4
    x = redc(lo_lo + hi * (R * R % p), p)
    return (x + reduce32(lo_hi, p)) % p


PW = 24


def eval_row(row, d, a, p):
    """Montgomery value of sum_i c_i a^i from Montgomery residues `row`
    (zero-padded to a multiple of 4), as the kernel computes it."""
    aM = mont(a, p)
    pw = [mont(1, p)]
    for _ in range(1, PW):
        pw.append(mmul(pw[-1], aM, p))
    apw = mmul(pw[-1], aM, p)
    if d < 0:
        return 0
    top = d // PW
    acc = 0
    for ch in range(top, -1, -1):
        ng = (min(PW, d + 1 - ch * PW) + 3) // 4
        S = 0
        for g in range(ng):
            t = sum(row[ch * PW + 4 * g + u] * pw[4 * g + u] for u in range(4))
            assert t < 1 << 64
            S += t
        r = fold96(S, p)
        acc = r if ch == top else (mmul(acc, apw, p) + r) % p
    return acc


def eliminate(A, B, a, b, lb, p, fused):
    if fused and a == b + 1:
        n1 = mneg(A[a], p)
        n2 = mneg(mdot2(lb, A[a - 1], n1, B[b - 1], p), p)
        l2, l1 = mmul(lb, lb, p), mmul(lb, n1, p)
        bp = B[0]
        A[0] = mdot2(l2, A[0], n2, bp, p)
        for t in range(1, b):
            y = B[t]
            A[t] = mdot3(l2, A[t], l1, bp, n2, y, p)
            bp = y
        return
    while a >= b:
        nla = mneg(A[a], p)
        s = a - b
        for t in range(s):
            A[t] = mmul(lb, A[t], p)
        for t in range(s, a):
            A[t] = mdot2(lb, A[t], nla, B[t - s], p)
        a -= 1


def mpow(x, e, p):
    r = mont(1, p)
    for _ in range(e):
        r = mmul(r, x, p)
    return r


def minv(x, p):
    return mpow(x, p - 2, p) if p < 100 else mont(pow(x * pow(R, -1, p) % p, p - 2, p), p)


def uni_resultant(A, B, m, n, p, fused=True):
    """Montgomery form of det Sylvester(A, B) with formal degrees m, n."""
    A, B = list(A), list(B)
    one = mont(1, p)
    if m == 0 and n == 0:
        return one
    a = m
    while a >= 0 and A[a] == 0:
        a -= 1
    b = n
    while b >= 0 and B[b] == 0:
        b -= 1
    if a < 0:
        return mpow(B[0], m, p) if n == 0 else 0
    if b < 0:
        return mpow(A[0], n, p) if m == 0 else 0
    if a < m and b < n:
        return 0
    num, den, neg = one, one, False
    if a < m:
        num, neg = mpow(B[n], m - a, p), (n * (m - a)) & 1 == 1
    elif b < n:
        num = mpow(A[m], n - b, p)
    if a < b:
        A, B, a, b = B, A, b, a
        neg ^= (a * b) & 1 == 1
    pfx = one
    # fast path of the kernel (one lane here): while each remainder has degree
    # exactly b - 1, the step's exponent bookkeeping is x = [b > 1] and
    # d = (1 - b)(a - b - 1)
    eliminated, lb_done = False, 0
    while fused and b > 0:
        lb = B[b]
        eliminate(A, B, a, b, lb, p, fused)
        if A[b - 1] == 0:
            eliminated, lb_done = True, lb
            break
        neg ^= (a * b) & 1 == 1
        pfx = mmul(pfx, mmul(lb, lb, p), p)
        if b > 1:
            den = mmul(den, pfx, p)
        d = (1 - b) * (a - b - 1)
        if d > 0:
            num = mmul(num, mpow(lb, d, p), p)
        elif d < 0:
            den = mmul(den, mpow(lb, -d, p), p)
        A, B, a, b = B, A, b, b - 1
    while b > 0:
        lb = lb_done if eliminated else B[b]
        if eliminated:
            eliminated = False
        else:
            eliminate(A, B, a, b, lb, p, fused)
        c = b - 1
        while c >= 0 and A[c] == 0:
            c -= 1
        if c < 0:
            return 0
        neg ^= (a * b) & 1 == 1
        pfx = mmul(pfx, mmul(lb, lb, p), p)
        x = b - max(c, 1)
        if x >= 1:
            den = mmul(den, mpow(pfx, x, p), p)
        d = a - c - (a - b + 1) * b + 2 * (b - 1)
        if d > 0:
            num = mmul(num, mpow(lb, d, p), p)
        elif d < 0:
            den = mmul(den, mpow(lb, -d, p), p)
        A, B, a, b = B, A, b, c
    num = mmul(num, mpow(B[0], a, p), p)
    r = mmul(num, minv(den, p), p)
    return mneg(r, p) if neg else r


@pytest.mark.parametrize("seed", range(4))
def test_power_dot_evaluation(seed):
    rng = random.Random(seed)
    for _ in range(150):
        p = rng.choice(PRIMES)
        a = rng.randrange(0, 8192)
        d = rng.randrange(-1, 80)
        c = [rng.randrange(p) if rng.random() > 0.3 else rng.choice([0, p - 1]) for _ in range(d + 1)]
        row = [mont(x, p) for x in c] + [0] * (4 * rng.randrange(1, 3) - (d + 1) % 4)
        ref = sum(ci * pow(a, i, p) for i, ci in enumerate(c)) % p
        assert eval_row(row, d, a, p) == mont(ref, p)


def test_fold_bound_at_extremes():
    for p in PRIMES:
        top = (p - 1) * (p - 1)
        S = 24 * top                         # the largest chunk sum
        assert fold96(S, p) == S * pow(R, -1, p) % p
        assert fold96(0, p) == 0


@pytest.mark.parametrize("fused", [False, True])
def test_euclid_matches_sylvester_determinant(fused):
    rng = random.Random(11 + fused)
    for _ in range(1500):
        p = rng.choice(PRIMES)
        m, n = rng.randint(0, 7), rng.randint(0, 7)
        f = [rng.randrange(p) if rng.random() > 0.3 else rng.choice([0, 1, p - 1]) for _ in range(m + 1)]
        g = [rng.randrange(p) if rng.random() > 0.3 else rng.choice([0, 1, p - 1]) for _ in range(n + 1)]
        if rng.random() < 0.2:
            f[-1] = 0
        if rng.random() < 0.2:
            g[-1] = 0
        ref = det_mod(sylvester(f, g), p) if m + n else 1
        got = uni_resultant([mont(x, p) for x in f], [mont(x, p) for x in g], m, n, p, fused)
        assert got == mont(ref, p), (f, g)


def test_model_catches_a_planted_mistake():
    # a wrong sign of a multiplier of the fused step must be caught
    rng = random.Random(5)
    p = PRIMES[0]
    bad = 0
    for _ in range(200):
        m = n = 4
        f = [rng.randrange(p) for _ in range(m + 1)]
        g = [rng.randrange(p) for _ in range(n + 1)]
        A, B = [mont(x, p) for x in f], [mont(x, p) for x in g]
        ref = mont(det_mod(sylvester(f, g), p), p)
        saved = globals()["mneg"]
        try:
            calls = {"k": 0}

            def flipped(x, q):
                calls["k"] += 1
                return x if calls["k"] % 2 == 0 else saved(x, q)

            globals()["mneg"] = flipped
            got = uni_resultant(A, B, m, n, p, True)
        finally:
            globals()["mneg"] = saved
        bad += got != ref
    assert bad > 150


def xcd_block(b, nb):
    q, r, x = nb >> 3, nb & 7, b & 7
    return x * q + min(x, r) + (b >> 3)


@pytest.mark.parametrize("nb", [1, 7, 8, 9, 63, 64, 65, 1000, 4096 * 49 + 5])
def test_xcd_block_map_is_a_bijection_with_contiguous_xcd_ranges(nb):
    logical = [xcd_block(b, nb) for b in range(nb)]
    assert sorted(logical) == list(range(nb))
    for x in range(8):
        mine = sorted(logical[b] for b in range(x, nb, 8))
        assert mine == list(range(mine[0], mine[0] + len(mine))) if mine else True


def _primes_desc(n):
    import sympy
    out, c = [], CEIL
    while len(out) < n:
        if sympy.isprime(c):
            out.append(c)
        c -= 2
    return out


def crt_model(residues, primes):
    """The explicit CRT of the limb kernel: y_k = x_k w_k mod p_k,
    t = nearest integer to sum y_k / p_k (fp64), R = sum y_k M_k - t M,
    assembled from signed 32-bit column sums with carries."""
    import math
    P = len(primes)
    M = math.prod(primes)
    LM = (M.bit_length() + 31) // 32
    Mk = [M // p for p in primes]
    y = [x * pow(mk % p, -1, p) % p for x, mk, p in zip(residues, Mk, primes)]
    f = 0.0
    for yk, p in zip(y, primes):
        f = math.fma(float(yk), 1.0 / p, f) if hasattr(math, "fma") else f + float(yk) * (1.0 / p)
    t = int(f + 0.5)
    limbs, carry = [], 0
    for l in range(LM):
        col = sum(yk * ((mk >> (32 * l)) & 0xFFFFFFFF) for yk, mk in zip(y, Mk))
        col -= t * ((M >> (32 * l)) & 0xFFFFFFFF)
        assert -(1 << 95) <= col < 1 << 95
        v = col + carry
        limbs.append(v & 0xFFFFFFFF)
        carry = v >> 32
    assert carry in (0, -1)
    val = sum(w << (32 * i) for i, w in enumerate(limbs))
    return val - (1 << (32 * LM)) if carry == -1 else val


def test_explicit_crt_at_the_margin():
    import math
    primes = _primes_desc(60)
    rng = random.Random(21)
    for P in (1, 2, 3, 7, 49, 60):
        ps = primes[:P]
        M = math.prod(ps)
        # the largest bound the planner admits for this P: M > 2^1.001 B
        from fractions import Fraction
        B = int(Fraction(M) * Fraction(2.0 ** -1.001)) - 1
        for R in [0, 1, -1, B, -B, B - 1, -B + 1] + [rng.randint(-B, B) for _ in range(40)]:
            assert crt_model([R % p for p in ps], ps) == R, (P, R)


# ---------------------------------------------------------------------------
# interpolation as a matrix product: coefficients = V^{-1} values, with V the
# Vandermonde matrix of the nodes 0..D-1, and V^{-1} by synthetic division:
# column a holds the coefficients of N(x) / ((x - a) N'(a)), N = prod (x - b).
# Products of residues are formed from balanced base-256 digits (int8) with
# 32-bit sums grouped by digit weight, as the int8 matrix-core kernel does.

def vinv_columns(D, p):
    N = [1]
    for b in range(D):                      # N <- N (x - b)
        N = [((N[j - 1] if j else 0) - b * (N[j] if j < len(N) else 0)) % p for j in range(len(N) + 1)]
    cols = []
    for a in range(D):
        q = [0] * D
        q[D - 1] = N[D]
        for j in range(D - 1, 0, -1):
            q[j - 1] = (N[j] + a * q[j]) % p
        fa = 1
        for b in range(D):
            if b != a:
                fa = fa * (a - b) % p
        w = pow(fa, p - 2, p)
        cols.append([w * qi % p for qi in q])
    return cols                              # cols[a][i] = V^{-1}[i][a]


def balanced_digits(x, p):
    v = x - p if x > p // 2 else x
    d = []
    for _ in range(3):
        r = ((v + 128) & 255) - 128
        d.append(r)
        v = (v - r) >> 8
    assert -128 <= v <= 127
    d.append(v)
    return d


def test_vinv_by_synthetic_division_inverts_vandermonde():
    p = PRIMES[1]
    for D in (1, 2, 5, 13):
        cols = vinv_columns(D, p)
        for i in range(D):
            for c in range(D):
                # (V^{-1} V)[i][c] = sum_a V^{-1}[i][a] a^c
                s = sum(cols[a][i] * pow(a, c, p) for a in range(D)) % p
                assert s == (1 if i == c else 0)


def test_packed_digits_by_offset_and_flip():
    # the kernels pack the four balanced digits of the symmetric representative
    # v as ((v + 0x808080) mod 2^32) xor 0x808080, one byte per digit
    rng = random.Random(5)
    for p in PRIMES + [3, 257, 65537]:
        for x in [0, 1, p - 1, p // 2, p // 2 + 1] + [rng.randrange(p) for _ in range(3000)]:
            v = x - p if x > p // 2 else x
            w = ((v + 0x808080) & 0xFFFFFFFF) ^ 0x808080
            got = [((w >> (8 * s)) & 255) - (256 if (w >> (8 * s)) & 128 else 0) for s in range(4)]
            assert got == balanced_digits(x, p), (x, p)


def test_digit_group_sums_stay_within_the_epilogue_bound():
    # seven weight groups of up to four int8 x int8 products per contraction
    # index, at most 4096 indices (padded D): |G_u| <= 2^28, and the signed sum
    # against residues below p < 2^32 / 3 stays inside 2^62 < p 2^32
    bound = 4 * 4096 * 128 * 128
    assert bound <= 1 << 28
    assert 7 * bound * ((1 << 32) // 3) < 1 << 62 < PRIMES[-1] * (1 << 32)


def test_digit_grouped_products_reconstruct_the_residue():
    rng = random.Random(8)
    for p in PRIMES:
        w = [pow(256, u, p) for u in range(7)]
        for _ in range(30):
            K = rng.randrange(1, 70)
            A = [rng.randrange(p) for _ in range(K)]
            B = [rng.randrange(p) for _ in range(K)]
            dA = [balanced_digits(x, p) for x in A]
            dB = [balanced_digits(x, p) for x in B]
            for x, d in zip(A, dA):
                assert sum(di << (8 * s) for s, di in enumerate(d)) % p == x
            G = [0] * 7
            for s in range(4):
                for t in range(4):
                    G[s + t] += sum(da[s] * db[t] for da, db in zip(dA, dB))
            assert all(abs(g) < 1 << 31 for g in G)
            got = sum((g % p) * wu for g, wu in zip(G, w)) % p
            assert got == sum(a * b for a, b in zip(A, B)) % p
            # the kernel's epilogue: signed sum against the Montgomery forms
            # of 256^u, offset by p 2^32, one reduction, one subtraction
            R = 1 << 32
            wm = [(pow(256, u, p) * R) % p for u in range(7)]
            t = sum(g * wu for g, wu in zip(G, wm))
            assert abs(t) < 1 << 62
            t += p * R
            assert 0 <= t < 2 * p * R
            pinv = (-pow(p, -1, R)) % R
            m = ((t % R) * pinv) % R
            u = t + m * p
            assert u < 1 << 64 and u % R == 0
            v = u >> 32
            v = v - p if v >= p else v
            v = v - p if v >= p else v
            assert v == got


def crt_model_mfma(residues, primes, Lc=None):
    """The matrix-core CRT: y_k as the symmetric representative of x_k w_k
    mod p_k, t = nearest integer to sum y_k / p_k (fp64), and X = sum_k y_k M_k
    formed as byte-column sums S_c = sum_{k,s} d_ks e_k(c - s) of balanced
    base-256 digits (d of y_k, e of M_k; the int8 product), folded into
    32-bit limbs of X - t M, eight per tile of 32 columns, with one signed
    carry; returns the two's-complement value of Lc limbs."""
    import math
    P = len(primes)
    M = math.prod(primes)
    LM = (M.bit_length() + 31) // 32
    NCT = (4 * LM + 4 + 31) // 32
    Mk = [M // p for p in primes]
    y = [x * pow(mk % p, -1, p) % p for x, mk, p in zip(residues, Mk, primes)]
    f = 0.0
    for yk, p in zip(y, primes):
        ys = yk - p if yk > p // 2 else yk
        f = math.fma(float(ys), 1.0 / p, f) if hasattr(math, "fma") else f + float(ys) * (1.0 / p)
    t = math.floor(f + 0.5)
    d = [balanced_digits(yk, p) for yk, p in zip(y, primes)]
    e = []
    for mk in Mk:
        dig, carry = [], 0
        for j in range(4 * LM):
            v = ((mk >> (8 * j)) & 255) + carry
            carry = 1 if v >= 128 else 0
            dig.append(v - 256 * carry)
        dig.append(carry)
        assert sum(di << (8 * j) for j, di in enumerate(dig)) == mk
        e.append(dig)
    S = [0] * (32 * NCT)
    for c in range(32 * NCT):
        for k in range(P):
            for s_ in range(4):
                if 0 <= c - s_ < 4 * LM + 1:
                    S[c] += d[k][s_] * e[k][c - s_]
        assert abs(S[c]) <= P * (3 * 128 + 64) * 128 < 1 << 23
    assert all(abs(dk[3]) <= 64 for dk in d)
    Lc = Lc or LM
    limbs, carry = [], 0
    for L in range(max(8 * NCT, Lc)):
        v = carry
        if L < 8 * NCT:
            lo, hi = S[4 * L] + (S[4 * L + 1] << 8), S[4 * L + 2] + (S[4 * L + 3] << 8)
            assert -(1 << 31) <= lo < 1 << 31 and -(1 << 31) <= hi < 1 << 31
            v += lo + (hi << 16)
        if L < LM:
            v -= t * ((M >> (32 * L)) & 0xFFFFFFFF)
        assert -(1 << 63) <= v < 1 << 63
        limbs.append(v & 0xFFFFFFFF)
        carry = v >> 32
    sign = limbs[Lc - 1] >> 31
    assert carry == (-1 if sign else 0)
    assert all(w == (0xFFFFFFFF if sign else 0) for w in limbs[Lc:])
    val = sum(w << (32 * i) for i, w in enumerate(limbs[:Lc]))
    return val - (1 << (32 * Lc)) if sign else val


def test_explicit_crt_on_digit_columns():
    import math
    from fractions import Fraction
    primes = _primes_desc(70)
    rng = random.Random(23)
    for P in (1, 2, 7, 17, 48, 70):
        ps = primes[:P]
        M = math.prod(ps)
        B = int(Fraction(M) * Fraction(2.0 ** -1.001)) - 1
        LM = (M.bit_length() + 31) // 32
        for R in [0, 1, -1, B, -B, B - 1] + [rng.randint(-B, B) for _ in range(12)]:
            for Lc in (LM, LM + 1, 8 * ((4 * LM + 35) // 32) + 3):
                assert crt_model_mfma([R % p for p in ps], ps, Lc=Lc) == R, (P, R, Lc)


def test_newton_block_tables_expand_the_newton_form():
    # The interpolation kernel's block tables: W_b[j][r] = [x^j] prod_{t<r}
    # (x - 32 b - t) and Q_b = prod_{t<32} (x - 32 b - t).  With T_b[j] =
    # sum_{r>=j} W_b[j][r] c_{32 b + r}, Horner over blocks (P <- P Q_b + T_b
    # from the top block down) must give the monomial coefficients of the
    # Newton form sum_k c_k prod_{t<k} (x - t) on the nodes 0, 1, 2, ...
    p = PRIMES[3]
    KB = 32
    rng = random.Random(77)

    def mul_lin(poly, t):  # poly * (x - t)
        out = [0] * (len(poly) + 1)
        for j, a in enumerate(poly):
            out[j + 1] = (out[j + 1] + a) % p
            out[j] = (out[j] - t * a) % p
        return out

    for D in (1, 5, 32, 33, 70, 97):
        c = [rng.randrange(p) for _ in range(D)]
        # direct Newton expansion
        ref, basis = [0] * D, [1]
        for k in range(D):
            for j, a in enumerate(basis):
                ref[j] = (ref[j] + c[k] * a) % p
            basis = mul_lin(basis, k)
        nb = -(-D // KB)
        T, Q = [], []
        for b in range(nb):
            N, W = [1], [[0] * KB for _ in range(KB)]
            for r in range(KB):
                for j, a in enumerate(N):
                    if j < KB:
                        W[j][r] = a
                N = mul_lin(N, KB * b + r)
            Q.append(N)
            length = min(KB, D - KB * b)
            T.append([sum(W[j][r] * c[KB * b + r] for r in range(j, length)) % p if j < length else 0
                      for j in range(KB)])
        P = T[nb - 1][:]
        for b in range(nb - 2, -1, -1):
            prod = [0] * (len(P) + KB)
            for i, a in enumerate(P):
                for t, qv in enumerate(Q[b]):
                    prod[i + t] = (prod[i + t] + a * qv) % p
            P = [(prod[j] + (T[b][j] if j < KB else 0)) % p for j in range(len(prod))]
        P = (P + [0] * D)[:D]
        assert P == ref, D


# ---------------------------------------------------------------------------
# principal subresultant coefficients per point (k_psc's psc_lane)

def psc_lane_model(A, B, m, n, K, p):
    """The kernel's recurrence for sr_0..sr_{K-1} of (A, B) with formal degrees
    (m, n), Montgomery inputs; returns plain values.  Same steps as psc_lane:
    closed-form top index, row-block exchange, formal drops, then Euclid with
    the scaled remainders' scalars tracked and one simultaneous inversion."""
    A, B = list(A), list(B)
    one = mont(1, p)
    num, den = [None] * K, [None] * K
    st = {"Nn": one, "Nd": one, "E0": 0, "E1": 0}

    def emit(i, vn, vd):
        if i >= K:
            return
        x = mmul(st["Nn"], vn, p)
        if (st["E0"] ^ (i & st["E1"])) & 1:
            x = mneg(x, p)
        assert num[i] is None, "index emitted twice"
        num[i], den[i] = x, mmul(st["Nd"], vd, p)

    def swap_sign(a, b):
        st["E0"] ^= (a * b) & 1
        st["E1"] ^= (a + b + 1) & 1

    a, b = m, n
    if a > b:
        emit(b, mpow(B[b], a - b, p), one)
    elif a < b:
        emit(a, mpow(A[a], b - a, p), one)
    if a < b:
        A, B, a, b = B, A, b, a
        swap_sign(a, b)
    while b >= 1:
        za, zb = A[a] == 0, B[b] == 0
        if not za and not zb:
            break
        if za and zb:
            for i in range(b):
                emit(i, 0, one)
            b = 0
            break
        if zb:
            st["Nn"] = mmul(st["Nn"], A[a], p)
            b -= 1
            emit(b, mpow(B[b], a - b, p), one)
            continue
        st["E0"] ^= b & 1
        st["E1"] ^= 1
        st["Nn"] = mmul(st["Nn"], B[b], p)
        a -= 1
        if a < b:
            A, B, a, b = B, A, b, a
            swap_sign(a, b)
            emit(b, mpow(B[b], a - b, p), one)
    sA = sB = one
    while b >= 1:
        lb = B[b]
        eliminate(A, B, a, b, lb, p, True)
        c = b - 1
        while c >= 0 and A[c] == 0:
            c -= 1
        for i in range(c + 1, b):
            emit(i, 0, one)
        if c < 0:
            break
        sR = mmul(mpow(lb, a - b + 1, p), sA, p)
        swap_sign(a, b)
        st["Nn"] = mmul(st["Nn"], mpow(lb, a - c, p), p)
        st["Nd"] = mmul(st["Nd"], mpow(sB, a - c, p), p)
        emit(c, mpow(A[c], b - c, p), mpow(sR, b - c, p))
        A, B, a, b, sA, sB = B, A, b, c, sB, sR
    assert all(v is not None for v in num), "index never emitted"
    pre = one
    for i in range(K):
        num[i] = mmul(num[i], pre, p)
        pre = mmul(pre, den[i], p)
    inv = minv(pre, p)
    out = [0] * K
    for i in reversed(range(K)):
        v = mmul(num[i], inv, p)
        inv = mmul(inv, den[i], p)
        out[i] = redc(v, p)
    return out


def _psc_det(fc, gc, p):
    from oracle.subresultants import psc_indices, psc_matrix
    m, n = len(fc) - 1, len(gc) - 1
    return [det_mod(psc_matrix(fc, gc, i), p) if m + n - 2 * i > 0 else 1 % p for i in psc_indices(m, n)]


def _psc_cases(rng, p):
    for _ in range(40):
        m, n = rng.randint(0, 7), rng.randint(0, 7)
        if m == n == 0:
            continue
        fc = [rng.randrange(p) for _ in range(m + 1)]
        gc = [rng.randrange(p) for _ in range(n + 1)]
        yield fc, gc
    # vanishing formal leading coefficients (one, several, both)
    yield [3, 1, 4, 0], [2, 7, 1]
    yield [3, 1, 0, 0], [2, 7, 1, 5]
    yield [3, 1, 4, 1], [2, 7, 0, 0]
    yield [3, 1, 4, 0], [2, 7, 1, 0]
    yield [5, 0, 0, 0, 0], [1, 2, 0]
    # common factors (defective sequences): (y - 2)^2 (y + 1) and (y - 2)^2
    yield [4, 0, -3 % p, 1], [4, -4 % p, 1]
    yield [(-8) % p, 12, -6 % p, 1], [4, -4 % p, 1]
    # a remainder that skips degrees: y^5 + 1 and y^2
    yield [1, 0, 0, 0, 0, 1], [0, 0, 1]


@pytest.mark.parametrize("p", [1431655751, 1073741827])
def test_psc_recurrence_matches_determinants(p):
    from oracle.subresultants import psc_indices
    rng = random.Random(p)
    for fc, gc in _psc_cases(rng, p):
        m, n = len(fc) - 1, len(gc) - 1
        K = len(psc_indices(m, n))
        got = psc_lane_model([mont(v, p) for v in fc], [mont(v, p) for v in gc], m, n, K, p)
        assert got == _psc_det(fc, gc, p), (fc, gc)


def test_psc_model_catches_a_planted_mistake():
    """Dropping the remainder's scalar (sR = 1) gives wrong values below the
    top two indices; the determinant comparison sees it."""
    p = 1431655751
    rng = random.Random(3)
    fc = [rng.randrange(p) for _ in range(6)]
    gc = [rng.randrange(p) for _ in range(5)]
    got = psc_lane_model([mont(v, p) for v in fc], [mont(v, p) for v in gc], 5, 4, 5, p)
    assert got == _psc_det(fc, gc, p)
    global mpow
    real = mpow
    try:
        mpow = lambda x, e, q: real(x, e, q) if e != 2 else real(x, 1, q)  # noqa: E731
        bad = psc_lane_model([mont(v, p) for v in fc], [mont(v, p) for v in gc], 5, 4, 5, p)
    finally:
        mpow = real
    assert bad != _psc_det(fc, gc, p)
