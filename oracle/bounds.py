"""A-priori size bounds of res(f, g; y), from the Sylvester matrix alone.

(Test infrastructure; see oracle/__init__.py.)  Both bounds are read off the
Sylvester matrix of Section 2 ("Resultants" paragraph) through the Leibniz
expansion det S = sum over permutations s of sign(s) * prod_i S[i][s(i)]:

* degree: every term has degree at most sum_i deg S[i][s(i)], so deg R is at
  most the largest such sum over permutations, a maximum-weight assignment on
  the matrix of entry degrees (zero entries are forbidden cells).  Section 2
  states the coarser deg R <= m*n for total degrees m and n.
* size: on |x| = 1 every entry is at most its 1-norm in absolute value, and
  |det| is at most the permanent of the absolute values, which is at most the
  product of the row sums.  Cauchy's estimate |c_i| <= max_{|x|=1} |R(x)| then
  bounds every coefficient of R by prod_rows sum_j ||S[i][j]||_1.

Together they say how many values of R at distinct nodes, and modulo how large
a number, fix R completely.
"""

from . import zx
from .resultant import bi_diff_y, bi_trim, sylvester


def _entries(F, G):
    F = bi_trim(F)
    G = bi_trim(G)
    if not F or not G:
        return None
    return sylvester(F, G)


def degree_bound(F, G):
    """Largest sum of entry degrees over the permutations of the Sylvester
    matrix of (f, g) in y; -1 when every permutation meets a zero entry (then
    det = 0).  The empty matrix (m_y = n_y = 0) has the bound 0 (det = 1)."""
    import numpy as np
    from scipy.optimize import linear_sum_assignment

    S = _entries(F, G)
    if S is None:
        return -1
    r = len(S)
    if r == 0:
        return 0
    forbid = -(10 ** 9)
    w = np.array([[zx.deg(e) if zx.trim(e) else forbid for e in row] for row in S], dtype=np.int64)
    rows, cols = linear_sum_assignment(w, maximize=True)
    total = int(w[rows, cols].sum())
    if any(w[i, j] == forbid for i, j in zip(rows, cols)):
        return -1
    return total


def coeff_bound(F, G):
    """prod over the Sylvester rows of the sum of the entries' 1-norms: an
    upper bound of |c_i| for every coefficient c_i of res(f, g; y)."""
    S = _entries(F, G)
    if S is None:
        return 0
    b = 1
    for row in S:
        b *= sum(sum(abs(c) for c in e) for e in row)
    return b


def discriminant_bounds(F):
    """(degree_bound, coeff_bound) of res(f, f_y; y)."""
    Fy = bi_diff_y(F)
    return degree_bound(F, Fy), coeff_bound(F, Fy)
