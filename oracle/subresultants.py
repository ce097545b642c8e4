"""Principal subresultant coefficients and the N^- / N^+ test.  (Test infrastructure; see oracle/__init__.py.)

Definitions followed (Section 3.2.2):

* "(Exact) Computation of N": the i-th subresultant Sres_i(f, g; y) of f, g
  with y-degrees m, n is the determinant of a Sylvester-like matrix with n - i
  shifted rows of f's y-coefficients and m - i shifted rows of g's, whose last
  column holds the polynomials y^k f and y^k g themselves.  Its coefficient of
  y^i is the i-th principal subresultant coefficient sr_i(x) in Z[x].  By
  linearity of the determinant in its last column, sr_i is the determinant of
  the same matrix with that column replaced by the coefficients of y^i: the
  first m + n - 2i columns of the coefficient matrix, entry (t, c) = f_{m-c+t}
  in the f-rows t < n - i and g_{n-c+t} in the g-rows t < m - i (indices
  outside 0..m or 0..n give 0).  sr_0 is the resultant of Section 2.
* The same paragraph: with R = res(f, f_y; y) and R* its square-free part,
  S_0 = R*, S_i = gcd(S_{i-1}, sr_i), R_i = S_{i-1} / S_i, d_i = deg R_i and
  N = sum_{i >= 1} (n_y - i) d_i (the gcds are nested, so the gcd of
  S_0, ..., S_i is S_i).  The paper's algorithm never computes this; the
  oracle does, to pin the bounds below.
* "Computation of N^-" (eq. lower-bound): the same chain over Z_p for one
  prime p, with sr_i^(p) the principal subresultant coefficients of f mod p
  and f_y mod p: N^- = sum_{i >= 1} (n_y - i) d_i^(p).
* "Computation of N^+" (eq. up-bound): N^+ = deg R* deg_y f - deg R +
  deg gcd(R^inf mod p, Q mod p), Q = res(f_x*, f_y*; y), where gcd(R^inf, Q)
  is the product of the common factors of R and Q with their multiplicity in
  Q.  Q is taken as res(f_x, f_y; y), the case gcd(f_x, f_y) = 1 (the
  remark after Teissier's lemma removes a common factor h first).

Readings where the paper is silent:
* Formal degrees.  m and n are the y-degrees of f and g as bivariate
  polynomials; sr_i^(p) is the reduction of the integer sr_i, i.e. the
  determinant keeps those formal degrees even where p divides a leading
  coefficient.  The lemma behind N^- assumes p divides neither lc_y f nor
  lc_y f_y; ``lower_bound`` reports such a prime as unlucky.
* Index range.  sr_i is formed for 0 <= i <= min(m, n), except i = m = n
  (a matrix with no rows).  For (f, f_y) that is i = 0 .. n_y - 1, and
  sr_{n_y-1} = n_y lc_y f.
"""

from . import zx
from .gcd import gcd_mod_p, gcd_zx
from .resultant import bi_diff_y, bi_trim, det_int, det_mod, det_zx, resultant_y


# ----------------------------------------------------------------------------
# the subresultant coefficient matrices

def psc_indices(m, n):
    """The indices i for which sr_i is formed (formal degrees m, n >= 0)."""
    top = min(m, n)
    return [i for i in range(top + 1) if not (i == m and i == n)]


def psc_matrix(fc, gc, i):
    """The (m+n-2i) x (m+n-2i) matrix whose determinant is sr_i.

    fc, gc list the y-coefficients in ascending order (entries are Z[x]
    polynomials or numbers); m = len(fc) - 1, n = len(gc) - 1 are the formal
    degrees.
    """
    m, n = len(fc) - 1, len(gc) - 1
    r = m + n - 2 * i
    zero = [] if (fc and isinstance(fc[0], list)) else 0
    M = [[zero] * r for _ in range(r)]
    for t in range(n - i):                  # f-rows
        for c in range(r):
            k = m - c + t
            if 0 <= k <= m:
                M[t][c] = fc[k]
    for t in range(m - i):                  # g-rows
        for c in range(r):
            k = n - c + t
            if 0 <= k <= n:
                M[n - i + t][c] = gc[k]
    return M


def _formal(F, G):
    F, G = bi_trim(F), bi_trim(G)
    if not F or not G:
        raise ValueError("subresultants of a zero polynomial are not formed")
    return F, G


def psc_zx(F, G):
    """[sr_i(x) for i in psc_indices(m, n)] in Z[x] (determinants over Z[x])."""
    F, G = _formal(F, G)
    m, n = len(F) - 1, len(G) - 1
    return [det_zx(psc_matrix(F, G, i)) for i in psc_indices(m, n)]


def psc_at(F, G, a):
    """[sr_i(a)] for an integer a (integer determinants of the specialised matrices)."""
    F, G = _formal(F, G)
    fa = [zx.evaluate(r, a) for r in F]
    ga = [zx.evaluate(r, a) for r in G]
    m, n = len(F) - 1, len(G) - 1
    return [det_int(psc_matrix(fa, ga, i)) for i in psc_indices(m, n)]


def psc_at_mod(F, G, a, p):
    """[sr_i(a) mod p] (determinants over F_p of the specialised matrices)."""
    F, G = _formal(F, G)
    fa = [zx.evaluate([c % p for c in r], a) % p for r in F]
    ga = [zx.evaluate([c % p for c in r], a) % p for r in G]
    m, n = len(F) - 1, len(G) - 1
    return [det_mod(psc_matrix(fa, ga, i), p) if m + n - 2 * i > 0 else 1 % p for i in psc_indices(m, n)]


# ----------------------------------------------------------------------------
# polynomials over F_p (ascending coefficient lists in 0..p-1, trimmed)

def fp(a, p):
    v = [c % p for c in a]
    while v and v[-1] == 0:
        v.pop()
    return v


def fp_deg(a):
    return len(a) - 1


def fp_divexact(a, b, p):
    """a / b over F_p; raises if b does not divide a."""
    a, b = fp(a, p), fp(b, p)
    if not b:
        raise ZeroDivisionError("division by the zero polynomial")
    inv = pow(b[-1], p - 2, p)
    r = list(a)
    q = [0] * max(0, len(a) - len(b) + 1)
    while len(r) >= len(b) and r:
        s = len(r) - len(b)
        t = r[-1] * inv % p
        q[s] = t
        for k, c in enumerate(b):
            r[s + k] = (r[s + k] - t * c) % p
        r = fp(r, p)
    if r:
        raise ArithmeticError("inexact division over F_p")
    return fp(q, p)


# ----------------------------------------------------------------------------
# the chain S_i of Section 3.2.2 and the two bounds

def chain_degrees(s0, srs, gcd):
    """deg S_0, deg S_1, ... with S_i = gcd(S_{i-1}, sr_i), until deg S_i = 0
    or the coefficients run out; ``gcd`` is the gcd of the ring."""
    degs = [len(s0) - 1]
    s = s0
    for sr in srs:
        if len(s) <= 1:
            break
        s = gcd(s, sr)
        degs.append(len(s) - 1)
    return degs


def count_from_degrees(ny, degs):
    """sum_{i >= 1} (n_y - i) d_i with d_i = n_{i-1} - n_i (n_i = 0 past the end)."""
    degs = list(degs)
    total = 0
    for i in range(1, len(degs) + 1):
        prev = degs[i - 1]
        cur = degs[i] if i < len(degs) else 0
        total += (ny - i) * (prev - cur)
    return total


def exact_count(F, Rstar):
    """N over Z: the chain with the integer psc's of (f, f_y) and gcds in Z[x]."""
    F = bi_trim(F)
    ny = len(F) - 1
    srs = psc_zx(F, bi_diff_y(F))
    return count_from_degrees(ny, chain_degrees(zx.trim(Rstar), srs[1:], gcd_zx))


def lower_bound_from_psc(ny, Rstar, srs_mod_p, p):
    """N^- (eq. lower-bound) from sr_1^(p), sr_2^(p), ... of (f, f_y) over F_p."""
    s0 = fp(Rstar, p)
    return count_from_degrees(ny, chain_degrees(s0, [fp(s, p) for s in srs_mod_p], lambda a, b: gcd_mod_p(a, b, p)))


def lucky(F, Rstar, p):
    """The lemma's condition on p: p divides neither lc_y f nor lc_y f_y (as
    polynomials in x), and deg (R* mod p) = deg R*."""
    F = bi_trim(F)
    fy = bi_diff_y(F)
    return bool(fp(F[-1], p)) and bool(fp(fy[-1], p)) and len(fp(Rstar, p)) == len(zx.trim(Rstar))


def lower_bound(F, Rstar, p):
    """N^- for a prime p, with the psc's of f mod p and f_y mod p."""
    F = bi_trim(F)
    srs = [fp(s, p) for s in psc_zx(F, bi_diff_y(F))]
    return lower_bound_from_psc(len(F) - 1, Rstar, srs[1:], p)


def bi_diff_x(F):
    """d/dx: row j of the result is the derivative of row j of F."""
    return bi_trim([zx.derivative(r) for r in bi_trim(F)])


def polar_resultant_y(F):
    """Q = res(f_x, f_y; y), the resultant of the remark after Teissier's lemma
    in the case gcd(f_x, f_y) = 1 (needs deg_y f >= 1)."""
    F = bi_trim(F)
    if len(F) < 2:
        raise ValueError("res(f_x, f_y; y) needs deg_y f >= 1")
    return resultant_y(bi_diff_x(F), bi_diff_y(F))


def common_part_degree_mod_p(R, Q, p):
    """deg gcd(R^inf mod p, Q mod p) over F_p."""
    r, q = fp(R, p), fp(Q, p)
    if not q:
        raise ValueError("Q vanishes mod p")
    total = 0
    while True:
        g = gcd_mod_p(q, r, p)
        if len(g) <= 1:
            return total
        total += len(g) - 1
        q = fp_divexact(q, g, p)


def common_part_degree_zx(R, Q):
    """deg gcd(R^inf, Q) over Z."""
    q = zx.trim(Q)
    total = 0
    while True:
        g = gcd_zx(q, R)
        if len(g) <= 1:
            return total
        total += len(g) - 1
        q = zx.exact_div(q, g)


def upper_bound(F, R, Rstar, Q, p):
    """N^+ (eq. up-bound) for a prime p."""
    ny = len(bi_trim(F)) - 1
    return (len(zx.trim(Rstar)) - 1) * ny - (len(zx.trim(R)) - 1) + common_part_degree_mod_p(R, Q, p)


def upper_bound_exact(F, R, Rstar, Q):
    """The sum of n_alpha^+ over the x-critical values (the lemma before eq. up-bound)."""
    ny = len(bi_trim(F)) - 1
    return (len(zx.trim(Rstar)) - 1) * ny - (len(zx.trim(R)) - 1) + common_part_degree_zx(R, Q)
