"""Pins of the subresultant / N^- / N^+ oracle against facts that do not come from it.

* sympy's subresultant sequence by Sylvester-submatrix determinants
  (``subresultants_sylv``) on pairs whose remainder sequence is complete: the
  leading coefficient of its element of degree i is sr_i;
* sr_0 = res(f, g; y), and sr_n = lc(g)^(m-n) for m > n (closed forms of the
  matrix);
* the characterisation the paper quotes in "(Exact) Computation of N":
  deg gcd(f(a,y), g(a,y)) = k iff sr_0(a) = ... = sr_{k-1}(a) = 0 != sr_k(a),
  by brute force over integer points with sympy's gcd;
* the exact count N against a count of distinct roots in each x-critical
  fiber, with the fiber's gcd taken over the algebraic number field of each
  irreducible factor of R* (sympy), and the sum of n_alpha^+ against sympy's
  factorisations of R and Q;
* the two lemmas: N^- <= N and N^+ >= sum n_alpha^+ >= N for several primes,
  with equality for primes that are not unlucky;
* Q = res(f_x, f_y; y) against sympy's Sylvester resultant of sympy's
  derivatives;
* a planted mistake in the psc matrix is caught by the sympy pin.
"""

import random

import pytest
import sympy as sp
from sympy.polys.subresultants_qq_zz import res as _sympy_sylvester_res
from sympy.polys.subresultants_qq_zz import subresultants_sylv

from oracle import zx
from oracle.resultant import bi_diff_y, bi_mul, bi_add, bi_trim, det_zx, resultant_y
from oracle.squarefree import squarefree_yun
from oracle.subresultants import (bi_diff_x, common_part_degree_mod_p, exact_count, fp, lower_bound, lucky,
                                  polar_resultant_y, psc_at, psc_at_mod, psc_indices, psc_matrix, psc_zx,
                                  upper_bound, upper_bound_exact)

X, Y = sp.symbols("x y")
PRIMES = [1000003, 998244353, 1431655751, 2147483647, 97, 101]


def to_sympy(F):
    return sum(c * X**i * Y**j for j, row in enumerate(F) for i, c in enumerate(row))


def from_sympy_x(e):
    if e == 0:
        return []
    p = sp.Poly(e, X)
    return zx.trim([int(c) for c in reversed(p.all_coeffs())])


def rand_curve(rng, t, lo=-3, hi=3):
    """Dense total degree t with a non-zero constant coefficient of y^t (so
    lc_y f is a constant: no vertical asymptote)."""
    F = [[rng.randint(lo, hi) for _ in range(t - j + 1)] for j in range(t + 1)]
    F[t][0] = F[t][0] or 1
    return F


def rand_uni(rng, d, lo=-9, hi=9):
    v = [rng.randint(lo, hi) for _ in range(d + 1)]
    v[-1] = v[-1] or 1
    return v


def as_rows(c):
    """A univariate polynomial in y with integer coefficients as a bivariate list."""
    return [[v] if v else [] for v in c]


def rstar(R):
    u, fs = squarefree_yun(R)
    out = [1]
    for a in fs:
        out = zx.mul(out, a)
    return out


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("seed", range(6))
def test_sr0_is_the_resultant(seed):
    rng = random.Random(seed)
    F, G = rand_curve(rng, rng.randint(1, 3)), rand_curve(rng, rng.randint(1, 3))
    assert psc_zx(F, G)[0] == resultant_y(F, G)


@pytest.mark.parametrize("seed", range(6))
def test_last_psc_is_a_power_of_lc(seed):
    rng = random.Random(100 + seed)
    m, n = rng.randint(2, 5), rng.randint(1, 4)
    if m <= n:
        m, n = n + 1, m
    fc, gc = rand_uni(rng, m), rand_uni(rng, n)
    srs = psc_zx(as_rows(fc), as_rows(gc))
    assert psc_indices(m, n)[-1] == n
    assert srs[-1] == zx.trim([gc[-1] ** (m - n)])
    # for (f, f_y): sr_{m-1} = m lc(f)
    fy = [(j + 1) * fc[j + 1] for j in range(m)]
    assert psc_zx(as_rows(fc), as_rows(fy))[-1] == zx.trim([m * fc[-1]])


# ---------------------------------------------------------------- library

def sympy_psc_complete(fc, gc):
    """sr_i from sympy's subresultant sequence, when it is complete."""
    f = sum(c * Y**j for j, c in enumerate(fc))
    g = sum(c * Y**j for j, c in enumerate(gc))
    seq = subresultants_sylv(f, g, Y)
    out = {}
    for s in seq[1:]:
        P = sp.Poly(s, Y)
        out[P.degree()] = int(P.LC())
    return out


@pytest.mark.parametrize("seed", range(10))
def test_matches_sympy_subresultant_sequence(seed):
    rng = random.Random(200 + seed)
    n = rng.randint(1, 4)
    m = n + rng.randint(0, 2)
    fc, gc = rand_uni(rng, m), rand_uni(rng, n)
    want = sympy_psc_complete(fc, gc)
    got = psc_zx(as_rows(fc), as_rows(gc))
    idx = psc_indices(m, n)
    # complete sequence: one element of every degree below n
    if sorted(d for d in want if d < n) != list(range(n)):
        pytest.skip("defective remainder sequence for this seed")
    for i, v in zip(idx, got):
        if i < n:
            assert zx.trim([want[i]]) == v, (i, want, got)


def test_planted_mistake_is_caught():
    """Swapping the f- and g-row counts (n-i rows of g, m-i of f) is a
    plausible slip; the sympy pin sees it."""
    def wrong_matrix(fc, gc, i):
        return psc_matrix(gc, fc, i)

    rng = random.Random(7)
    caught = False
    for _ in range(5):
        fc, gc = rand_uni(rng, 4), rand_uni(rng, 2)
        want = sympy_psc_complete(fc, gc)
        for i in (0, 1):
            if i in want:
                v = det_zx(wrong_matrix(as_rows(fc), as_rows(gc), i))
                caught |= v != zx.trim([want[i]])
    assert caught


# ---------------------------------------------------------------- brute force

def _curve_with_fiber_structure(rng):
    # f and g sharing factors above chosen points: g = f_y of a singular curve,
    # plus a pair with a common component at y = x
    a = [[rng.randint(-2, 2) for _ in range(3 - j)] for j in range(3)]
    b = [[rng.randint(-2, 2) for _ in range(2 - j)] for j in range(2)]
    a[-1] = [1]
    b[-1] = [1]
    lin = [[0, -1], [1]]  # y - x
    return bi_mul(lin, bi_mul(lin, a)), bi_mul(lin, b)


@pytest.mark.parametrize("seed", range(6))
def test_gcd_degree_characterisation(seed):
    rng = random.Random(300 + seed)
    if seed % 2:
        F, G = _curve_with_fiber_structure(rng)
    else:
        F = bi_add(bi_mul(rand_curve(rng, 2, -2, 2), rand_curve(rng, 1, -2, 2)), [[0, 0, 1]])
        G = bi_diff_y(F)
    F, G = bi_trim(F), bi_trim(G)
    m, n = len(F) - 1, len(G) - 1
    idx = psc_indices(m, n)
    for a in range(-6, 7):
        fa = sum(zx.evaluate(r, a) * Y**j for j, r in enumerate(F))
        ga = sum(zx.evaluate(r, a) * Y**j for j, r in enumerate(G))
        if sp.Poly(fa, Y).degree() != m or sp.Poly(ga, Y).degree() != n:
            continue  # the characterisation is for non-vanishing leading coefficients
        k = sp.Poly(sp.gcd(fa, ga), Y).degree()
        vals = psc_at(F, G, a)
        first_nonzero = next(i for i, v in zip(idx, vals) if v != 0)
        assert first_nonzero == k, (a, k, vals)


@pytest.mark.parametrize("seed", range(4))
def test_specialisations(seed):
    rng = random.Random(400 + seed)
    F, G = rand_curve(rng, 3), rand_curve(rng, 2)
    srs = psc_zx(F, G)
    for a in (-2, 0, 3):
        assert psc_at(F, G, a) == [zx.evaluate(s, a) for s in srs]
        for p in (97, 1000003):
            assert psc_at_mod(F, G, a, p) == [zx.evaluate(s, a) % p for s in srs]


# ---------------------------------------------------------------- N, N^-, N^+

def fiber_counts(F, max_factor_degree=0):
    """(N, sum n_alpha^+) from sympy: for each irreducible factor phi of R*,
    n_alpha = n_y - deg gcd(f(alpha, y), f_y(alpha, y)) over Q(alpha), and
    n_alpha^+ = n_y - mult(phi, R) + mult(phi, Q)."""
    f = to_sympy(F)
    ny = sp.Poly(f, Y).degree()
    fy, fx = sp.diff(f, Y), sp.diff(f, X)
    R = sp.Poly(f, Y).resultant(sp.Poly(fy, Y))
    Q = sp.Poly(fx, Y).resultant(sp.Poly(fy, Y))
    rfac = dict((sp.Poly(p, X), e) for p, e in sp.factor_list(R.as_expr(), X)[1] if sp.Poly(p, X).degree() > 0)
    if max_factor_degree and max(phi.degree() for phi in rfac) > max_factor_degree:
        return None
    qfac = dict((sp.Poly(p, X), e) for p, e in sp.factor_list(Q.as_expr(), X)[1] if sp.Poly(p, X).degree() > 0)
    N = Nplus = 0
    for phi, e in rfac.items():
        a = sp.CRootOf(phi, 0)
        K = sp.QQ.algebraic_field(a)
        g = sp.Poly(f.subs(X, a), Y, domain=K).gcd(sp.Poly(fy.subs(X, a), Y, domain=K))
        d = phi.degree()
        N += d * (ny - g.degree())
        mq = next((qe for qp, qe in qfac.items() if qp.monic() == phi.monic()), 0)
        Nplus += d * (ny - e + mq)
    return N, Nplus


CURVES = {
    # square-free curves without vertical asymptotes
    "cusp_and_node": [[0, 0, 0, -1], [], [1]],                    # y^2 - x^3
    "node": [[0, 0, -1, -1], [], [1]],                             # y^2 - x^2 - x^3
    "cubic": [[-2, 0, 0, 1], [0, -3], [], [1]],                    # y^3 - 3xy + x^3 - 2
    "quartic": [[0, 0, 0, 0, -1], [], [-2], [], [1]],             # y^4 - 2y^2 - x^4
}


@pytest.mark.parametrize("name", sorted(CURVES))
def test_exact_count_against_fibers(name):
    F = bi_trim(CURVES[name])
    R = resultant_y(F, bi_diff_y(F))
    Q = polar_resultant_y(F)
    N, Nplus = fiber_counts(F)
    assert exact_count(F, rstar(R)) == N
    assert upper_bound_exact(F, R, rstar(R), Q) == Nplus
    assert Nplus >= N


@pytest.mark.parametrize("seed", range(8))
def test_exact_count_random_curves(seed):
    rng = random.Random(500 + seed)
    # singular by construction: f = g^2 + h k^2 has singular points at g = k = 0
    g, h, k = rand_curve(rng, 1, -2, 2), rand_curve(rng, 1, -2, 2), rand_curve(rng, 1, -2, 2)
    F = bi_add(bi_mul(g, g), bi_mul(h, bi_mul(k, k)))
    F = bi_trim(F)
    R = resultant_y(F, bi_diff_y(F))
    if not R or len(bi_trim(F)[-1]) != 1:
        pytest.skip("vertical asymptote or non-square-free curve for this seed")
    counts = fiber_counts(F, max_factor_degree=4)
    if counts is None:
        pytest.skip("an x-critical factor of degree above 4 (sympy's algebraic gcd is slow there)")
    N, Nplus = counts
    assert exact_count(F, rstar(R)) == N
    assert upper_bound_exact(F, R, rstar(R), polar_resultant_y(F)) == Nplus


@pytest.mark.parametrize("name", sorted(CURVES))
def test_bounds_for_several_primes(name):
    F = bi_trim(CURVES[name])
    R = resultant_y(F, bi_diff_y(F))
    Rs = rstar(R)
    Q = polar_resultant_y(F)
    N = exact_count(F, Rs)
    Nsum = upper_bound_exact(F, R, Rs, Q)
    for p in PRIMES:
        if not lucky(F, Rs, p) or not fp(Q, p):
            continue
        lo = lower_bound(F, Rs, p)
        hi = upper_bound(F, R, Rs, Q, p)
        assert lo <= N <= Nsum <= hi, (p, lo, N, Nsum, hi)
        if p > 1000:
            assert lo == N and hi == Nsum


def test_small_prime_can_be_unlucky_but_stays_a_bound():
    # y^2 - x^3 - 7x: its critical values differ mod 7 only by a repeated root
    F = bi_trim([[0, -7, 0, -1], [], [1]])
    R = resultant_y(F, bi_diff_y(F))
    Rs = rstar(R)
    Q = polar_resultant_y(F)
    N = exact_count(F, Rs)
    for p in (3, 5, 7, 11, 13):
        if lucky(F, Rs, p) and fp(Q, p):
            assert lower_bound(F, Rs, p) <= N <= upper_bound(F, R, Rs, Q, p)


def test_common_part_degree_counts_multiplicity_in_q():
    # R = x^2 (x-1), Q = x^3 (x-1)^2 (x+1): common factors x^3 (x-1)^2 -> 5
    R = zx.mul([0, 0, 1], [-1, 1])
    Q = zx.mul(zx.mul([0, 0, 0, 1], zx.mul([-1, 1], [-1, 1])), [1, 1])
    assert common_part_degree_mod_p(R, Q, 1000003) == 5


# ---------------------------------------------------------------- Q

@pytest.mark.parametrize("seed", range(6))
def test_polar_resultant_matches_sympy(seed):
    rng = random.Random(600 + seed)
    F = rand_curve(rng, rng.randint(2, 4))
    f = to_sympy(F)
    want = from_sympy_x(sp.expand(_sympy_sylvester_res(sp.diff(f, X), sp.diff(f, Y), Y)))
    assert polar_resultant_y(F) == want


def test_diff_x_against_sympy():
    rng = random.Random(9)
    F = rand_curve(rng, 4)
    d = sp.Poly(sp.diff(to_sympy(F), X), X, Y)
    want = {(i, j): int(c) for (i, j), c in zip(d.monoms(), d.coeffs())}
    got = {(i, j): c for j, r in enumerate(bi_diff_x(F)) for i, c in enumerate(r) if c}
    assert got == want
