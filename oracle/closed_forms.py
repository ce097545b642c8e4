"""Inputs with a resultant known in closed form.  (Test infrastructure; see oracle/__init__.py.)

These are classical identities of the resultant over an integral domain
(Z[x] here), used as pins that do not go through a determinant:

* product form: for f = A(x) prod_i (y - a_i(x)) and g = B(x) prod_j (y - b_j(x)),
  res(f, g; y) = A^n B^m prod_{i,j} (a_i - b_j)   (m, n the numbers of roots);
* discriminant form: for f = A(x) prod_i (y - a_i(x)),
  res(f, f_y; y) = A^{2m-1} prod_{i != j} (a_i - a_j);
* linear f = f_1 y + f_0: res(f, g; y) = sum_j g_j (-f_0)^j f_1^{n-j};
* f free of y (m_y = 0): res(f, g; y) = f_0^{n_y}.

Theorem 1 (thm:resultants) ties the roots of R^{(y)} to common roots; the
product form is its quantitative version.
"""

from . import zx
from .resultant import bi_trim


def _prod_linear(lead, roots):
    """lead(x) * prod (y - r(x)) as a bivariate row list."""
    F = [list(lead)]
    for r in roots:
        # multiply F by (y - r): new[j] = F[j-1] - r*F[j]
        new = [[] for _ in range(len(F) + 1)]
        for j, row in enumerate(F):
            new[j + 1] = zx.add(new[j + 1], row)
            new[j] = zx.sub(new[j], zx.mul(r, row))
        F = new
    return bi_trim(F)


def product_pair(A, a_roots, B, b_roots):
    """(f, g, R) for f = A prod (y - a_i), g = B prod (y - b_j)."""
    f = _prod_linear(A, a_roots)
    g = _prod_linear(B, b_roots)
    m, n = len(a_roots), len(b_roots)
    R = zx.mul(zx.power(A, n), zx.power(B, m))
    for a in a_roots:
        for b in b_roots:
            R = zx.mul(R, zx.sub(a, b))
    return f, g, R


def product_discriminant(A, roots):
    """(f, R) for f = A prod (y - a_i) and R = res(f, f_y; y)."""
    f = _prod_linear(A, roots)
    m = len(roots)
    R = zx.power(A, 2 * m - 1)
    for i, a in enumerate(roots):
        for j, b in enumerate(roots):
            if i != j:
                R = zx.mul(R, zx.sub(a, b))
    return f, R


def linear_resultant(f1, f0, G):
    """res(f1 y + f0, g; y) = sum_j g_j (-f0)^j f1^(n-j)."""
    G = bi_trim(G)
    n = len(G) - 1
    R = []
    mf0 = zx.neg(f0)
    for j, gj in enumerate(G):
        R = zx.add(R, zx.mul(gj, zx.mul(zx.power(mf0, j), zx.power(f1, n - j))))
    return R
