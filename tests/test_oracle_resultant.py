"""Pins of the resultant oracle against facts that do not come from the oracle.

Each test names the fact it checks:
* a library routine (sympy's resultant) on tiny inputs;
* closed forms (product of root differences, discriminant, linear f, y-free f);
* invariants (antisymmetry, multiplicativity, scaling, y-shift);
* the evaluation homomorphism R(a) = det S(f(a,y), g(a,y)) with an independent
  rational Gaussian elimination;
* Theorem 1 (thm:resultants) by brute force on tiny inputs;
* the degree bound of Section 2 ("Resultants": deg R <= m n) and the sharper
  weighted bound used to size the interpolation.
"""

import random
from fractions import Fraction

import pytest
import sympy as sp
from sympy.polys.subresultants_qq_zz import res as _sympy_sylvester_res

from oracle import zx
from oracle.resultant import (bi_diff_y, bi_mul, bi_tdeg, bi_transpose, bi_trim, bi_ydeg,
                              det_int, det_mod, discriminant_y, resultant_at, resultant_at_mod,
                              resultant_x, resultant_y, sylvester)
from oracle.closed_forms import linear_resultant, product_discriminant, product_pair
from paper_1201_1548_amd import synth

X, Y = sp.symbols("x y")


def to_sympy(F):
    return sum(c * X**i * Y**j for j, row in enumerate(F) for i, c in enumerate(row))


def sympy_res_y(F, G):
    # sympy's own Sylvester-matrix resultant (its top-level ``resultant`` returns
    # the opposite sign for some degree pairs, e.g. (m_y, n_y) = (1, 3)).
    r = sp.Poly(_sympy_sylvester_res(to_sympy(F), to_sympy(G), Y), X)
    return zx.trim([int(c) for c in reversed(r.all_coeffs())]) if r.as_expr() != 0 else []


def small_pair(rng, tf, tg, lo=-3, hi=3):
    def one(t):
        return [[rng.randint(lo, hi) for _ in range(t - j + 1)] for j in range(t + 1)]
    F, G = one(tf), one(tg)
    F[-1][0] = F[-1][0] or 1
    G[-1][0] = G[-1][0] or 1
    return F, G


def rand_zx(rng, d, lo=-4, hi=4):
    return zx.trim([rng.randint(lo, hi) for _ in range(d + 1)]) or [1]


# ---------------------------------------------------------------- library

@pytest.mark.parametrize("seed", range(12))
def test_matches_sympy_resultant(seed):
    rng = random.Random(seed)
    F, G = small_pair(rng, rng.randint(1, 3), rng.randint(1, 3))
    assert resultant_y(F, G) == sympy_res_y(F, G)


@pytest.mark.parametrize("seed", range(4))
def test_matches_sympy_on_deg6_shape(seed):
    F, G = synth.pair_deg6(seed)
    F = [r[:4] for r in F[:4]]  # tdeg-6 rows cut to a 4x4 block keeps sympy fast
    G = [r[:4] for r in G[:4]]
    assert resultant_y(F, G) == sympy_res_y(F, G)


def test_sylvester_layout_matches_paper_display():
    # Section 2: first n_y rows shifted copies of f_m..f_0, then m_y rows of g_n..g_0.
    S = sylvester([1, 2, 3], [4, 5])   # f = 3y^2+2y+1, g = 5y+4
    assert S == [[3, 2, 1], [5, 4, 0], [0, 5, 4]]


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("seed", range(6))
def test_product_form(seed):
    rng = random.Random(100 + seed)
    m, n = rng.randint(1, 4), rng.randint(1, 4)
    A, B = rand_zx(rng, rng.randint(0, 2)), rand_zx(rng, rng.randint(0, 2))
    a = [rand_zx(rng, rng.randint(0, 2)) for _ in range(m)]
    b = [rand_zx(rng, rng.randint(0, 2)) for _ in range(n)]
    f, g, R = product_pair(A, a, B, b)
    assert resultant_y(f, g) == R


def test_product_form_common_root_vanishes():
    f, g, R = product_pair([2], [[1, 1], [3]], [1, 1], [[0, 5], [1, 1]])
    assert R == [] and resultant_y(f, g) == []


@pytest.mark.parametrize("seed", range(5))
def test_discriminant_closed_form(seed):
    rng = random.Random(200 + seed)
    m = rng.randint(2, 5)
    A = rand_zx(rng, rng.randint(0, 2))
    roots = [rand_zx(rng, rng.randint(0, 2)) for _ in range(m)]
    f, R = product_discriminant(A, roots)
    assert discriminant_y(f) == R


def test_discriminant_repeated_root_is_zero():
    f, R = product_discriminant([1, 2], [[1, 1], [1, 1], [0, 3]])
    assert R == [] and discriminant_y(f) == []


@pytest.mark.parametrize("seed", range(5))
def test_linear_f_closed_form(seed):
    rng = random.Random(300 + seed)
    f1, f0 = rand_zx(rng, 2), rand_zx(rng, 3)
    G = [[rng.randint(-5, 5) for _ in range(rng.randint(1, 4))] for _ in range(rng.randint(2, 5))]
    G[-1][0] = G[-1][0] or 2
    assert resultant_y([f0, f1], G) == linear_resultant(f1, f0, G)


def test_y_free_f_and_edge_conventions():
    f0 = [3, -1, 2]
    G = [[1, 2], [0, 1], [5]]
    assert resultant_y([f0], G) == zx.power(f0, 2)
    assert resultant_y([f0], [[7, 1]]) == [1]          # empty determinant
    assert resultant_y([], G) == [] and resultant_y(G, []) == []
    assert discriminant_y([[1, 2], [3, 4]]) == [3, 4]   # m_y = 1: res(f1 y + f0, f1) = f1
    with pytest.raises(ValueError):
        discriminant_y([[1, 2, 3]])


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", range(5))
def test_antisymmetry(seed):
    rng = random.Random(400 + seed)
    F, G = small_pair(rng, rng.randint(1, 4), rng.randint(1, 4))
    m, n = bi_ydeg(F), bi_ydeg(G)
    assert resultant_y(G, F) == zx.scale(resultant_y(F, G), (-1) ** (m * n))


@pytest.mark.parametrize("seed", range(4))
def test_multiplicativity(seed):
    rng = random.Random(500 + seed)
    F1, G = small_pair(rng, rng.randint(1, 3), rng.randint(1, 3))
    F2, _ = small_pair(rng, rng.randint(1, 2), 1)
    assert resultant_y(bi_mul(F1, F2), G) == zx.mul(resultant_y(F1, G), resultant_y(F2, G))


@pytest.mark.parametrize("seed", range(4))
def test_scaling(seed):
    rng = random.Random(600 + seed)
    F, G = small_pair(rng, rng.randint(1, 3), rng.randint(1, 3))
    c = rng.choice([-3, 2, 5])
    cF = [zx.scale(r, c) for r in F]
    assert resultant_y(cF, G) == zx.scale(resultant_y(F, G), c ** bi_ydeg(G))


@pytest.mark.parametrize("seed", range(3))
def test_y_shift_invariance(seed):
    rng = random.Random(700 + seed)
    F, G = small_pair(rng, rng.randint(1, 3), rng.randint(1, 3))
    s = rand_zx(rng, 1)
    shift = [s, [1]]                       # y -> y + s(x)

    def compose(P):
        out = []
        powr = [[1]]
        for row in P:
            out = _bi_add(out, bi_mul([row], powr))
            powr = bi_mul(powr, shift)
        return out

    assert resultant_y(compose(F), compose(G)) == resultant_y(F, G)


def _bi_add(A, B):
    n = max(len(A), len(B))
    return bi_trim([zx.add(A[j] if j < len(A) else [], B[j] if j < len(B) else []) for j in range(n)])


def test_res_x_is_res_y_of_transpose_and_sympy():
    rng = random.Random(42)
    F, G = small_pair(rng, 3, 2)
    rx = resultant_x(F, G)
    r = sp.Poly(_sympy_sylvester_res(to_sympy(F), to_sympy(G), X), Y)
    assert rx == zx.trim([int(c) for c in reversed(r.all_coeffs())])
    assert resultant_y(bi_transpose(F), bi_transpose(G)) == rx


# ---------------------------------------------------------------- specialisation

def _det_fraction(M):
    """Independent determinant: Gaussian elimination over Q."""
    A = [[Fraction(v) for v in row] for row in M]
    n = len(A)
    d = Fraction(1)
    for k in range(n):
        p = next((i for i in range(k, n) if A[i][k] != 0), None)
        if p is None:
            return 0
        if p != k:
            A[k], A[p] = A[p], A[k]
            d = -d
        d *= A[k][k]
        for i in range(k + 1, n):
            t = A[i][k] / A[k][k]
            for j in range(k, n):
                A[i][j] -= t * A[k][j]
    assert d.denominator == 1
    return int(d)


@pytest.mark.parametrize("seed", range(3))
def test_evaluation_homomorphism(seed):
    F, G = synth.pair_deg6(seed)
    R = resultant_y(F, G)
    for a in (-3, 0, 1, 7, 123456789):
        fa = [zx.evaluate(r, a) for r in F]
        ga = [zx.evaluate(r, a) for r in G]
        v = _det_fraction(sylvester(fa, ga))
        assert zx.evaluate(R, a) == v == resultant_at(F, G, a)
        q = 2147483647
        assert resultant_at_mod(F, G, a, q) == v % q


def test_det_helpers_agree_with_rational_elimination():
    rng = random.Random(9)
    for n in range(1, 7):
        M = [[rng.randint(-50, 50) for _ in range(n)] for _ in range(n)]
        v = _det_fraction(M)
        assert det_int(M) == v
        assert det_mod(M, 1000003) == v % 1000003


# ---------------------------------------------------------------- Theorem 1

def test_theorem1_brute_force():
    """R(a) = 0  <=>  f(a,y), g(a,y) share a root, or both leading coefficients vanish at a."""
    rng = random.Random(77)
    checked_zero = checked_nonzero = 0
    for _ in range(60):
        F, G = small_pair(rng, 2, 2, -2, 2)
        F[-1] = [rng.randint(-1, 1), rng.randint(-1, 1)]   # let lc_y vanish at some a
        G[-1] = [rng.randint(-1, 1), 1]
        if not bi_trim(F) or bi_ydeg(F) < 1:
            continue
        R = resultant_y(F, G)
        for a in range(-4, 5):
            fa = sp.Poly([zx.evaluate(r, a) for r in reversed(bi_trim(F))], Y)
            ga = sp.Poly([zx.evaluate(r, a) for r in reversed(bi_trim(G))], Y)
            lcs_vanish = zx.evaluate(bi_trim(F)[-1], a) == 0 and zx.evaluate(bi_trim(G)[-1], a) == 0
            common = sp.gcd(fa, ga).degree() > 0 if not (fa.is_zero or ga.is_zero) else True
            vanish = zx.evaluate(R, a) == 0
            assert vanish == (common or lcs_vanish)
            checked_zero += vanish
            checked_nonzero += not vanish
    assert checked_zero > 5 and checked_nonzero > 50


# ---------------------------------------------------------------- degree bounds

@pytest.mark.parametrize("seed", range(4))
def test_degree_bounds(seed):
    rng = random.Random(800 + seed)
    F, G = small_pair(rng, rng.randint(1, 4), rng.randint(1, 4))
    R = resultant_y(F, G)
    m, n = bi_ydeg(F), bi_ydeg(G)
    tf, tg = bi_tdeg(F), bi_tdeg(G)
    assert zx.deg(R) <= tf * tg
    assert zx.deg(R) <= n * tf + m * tg - m * n


def test_deg6_dense_degree_is_bezout():
    F, G = synth.pair_deg6(0)
    assert zx.deg(resultant_y(F, G)) == 36


# ---------------------------------------------------------------- planted mistakes

def test_pins_catch_planted_mistakes(monkeypatch):
    """A wrong oracle must fail a pin: plant typical mistakes and check they are caught."""
    import oracle.resultant as R

    rng = random.Random(5)
    F, G = small_pair(rng, 2, 3)
    good = sympy_res_y(F, G)
    orig = R.sylvester

    def g_rows_reversed(fc, gc):       # g coefficients written low-to-high
        return orig(fc, list(reversed(gc)))

    def rows_swapped(fc, gc):          # g block first: sign error when m*n odd
        S = orig(fc, gc)
        n = len(gc) - 1
        return S[n:] + S[:n]

    def wrong_shift(fc, gc):           # forgets to shift one row
        S = orig(fc, gc)
        S[1] = S[0][:]
        return S

    F2, G2 = small_pair(random.Random(6), 1, 3)   # m*n = 3 odd for the block swap
    for bad, (ff, gg) in ((g_rows_reversed, (F, G)), (rows_swapped, (F2, G2)), (wrong_shift, (F, G))):
        monkeypatch.setattr(R, "sylvester", bad)
        assert R.resultant_y(ff, gg) != sympy_res_y(ff, gg)
        monkeypatch.setattr(R, "sylvester", orig)
    assert R.resultant_y(F, G) == good
