"""Resultants over Z[x] by the plain definition.  (Test infrastructure; see oracle/__init__.py.)

Bivariate polynomials are lists of rows: ``F[j]`` is the Z[x] polynomial
f_j^{(y)}(x) (ascending powers of x) multiplying y^j, i.e. ``F[j][i]`` is the
coefficient of x^i y^j.  m_y is the index of the last non-zero row (the degree
of f in y, Section 2, "Notation").

Definition followed (Section 2, "Resultants" paragraph): R^{(y)} = res(f, g; y)
is the determinant of the (m_y+n_y) x (m_y+n_y) Sylvester matrix whose first
n_y rows hold shifted copies of f's y-coefficients from f_{m_y} down to f_0 and
whose last m_y rows hold shifted copies of g's.  res(f, g; x) is the same with
the variables exchanged.  The curve-analysis resultant of Section 3.1 (Project)
is res(f, f_y; y).

Conventions the paper leaves open (each is listed in the design notes):
* f = 0 or g = 0 gives R = 0;
* m_y = n_y = 0 gives the empty determinant, R = 1;
* m_y = 0 < n_y gives R = f_0^{n_y} (the matrix is f_0 times the identity);
* res(f, f_y; y) is returned as is: no division by the leading coefficient
  and no (-1)^{m(m-1)/2} sign; it needs m_y >= 1.
"""

from . import zx


# ----------------------------------------------------------------------------
# bivariate helpers (plain data manipulation)

def bi_trim(F):
    rows = [zx.trim(r) for r in F]
    while rows and not rows[-1]:
        rows.pop()
    return rows


def bi_ydeg(F):
    return len(bi_trim(F)) - 1


def bi_xdeg(F):
    return max((len(r) - 1 for r in bi_trim(F) if r), default=-1)


def bi_tdeg(F):
    F = bi_trim(F)
    return max((i + j for j, r in enumerate(F) for i, c in enumerate(r) if c), default=-1)


def bi_transpose(F):
    """Exchange x and y: the result's row i holds the coefficients of x^i."""
    F = bi_trim(F)
    nx = bi_xdeg(F) + 1
    return bi_trim([[F[j][i] if i < len(F[j]) else 0 for j in range(len(F))] for i in range(nx)])


def bi_diff_y(F):
    """d/dy: row j of the result is (j+1) * row j+1 of F."""
    F = bi_trim(F)
    return bi_trim([zx.scale(F[j], j) for j in range(1, len(F))])


def bi_add(F, G):
    n = max(len(F), len(G))
    return bi_trim([zx.add(F[j] if j < len(F) else [], G[j] if j < len(G) else []) for j in range(n)])


def bi_mul(F, G):
    F = bi_trim(F)
    G = bi_trim(G)
    if not F or not G:
        return []
    out = [[] for _ in range(len(F) + len(G) - 1)]
    for j, a in enumerate(F):
        for k, b in enumerate(G):
            out[j + k] = zx.add(out[j + k], zx.mul(a, b))
    return bi_trim(out)


def bi_eval_x(F, a):
    """f(a, y) as a list of y-coefficients (ints), untrimmed: length m_y+1."""
    return [zx.evaluate(r, a) for r in bi_trim(F)]


# ----------------------------------------------------------------------------
# Sylvester matrix and determinants

def sylvester(fc, gc):
    """Sylvester matrix of Section 2 for coefficient lists fc, gc (ascending in y).

    Entries are whatever objects the lists hold (Z[x] polynomials or numbers);
    zero entries are the ``zero`` of the entry type (``[]`` for polynomials).
    """
    m = len(fc) - 1
    n = len(gc) - 1
    r = m + n
    zero = [] if fc and isinstance(fc[0], list) else 0
    S = [[zero] * r for _ in range(r)]
    for t in range(n):                      # f-rows: f_m, f_{m-1}, ..., f_0
        for s in range(m + 1):
            S[t][t + s] = fc[m - s]
    for t in range(m):                      # g-rows: g_n, ..., g_0
        for s in range(n + 1):
            S[n + t][t + s] = gc[n - s]
    return S


def det_zx(M):
    """Determinant over Z[x] by fraction-free (Bareiss) elimination.

    Each update a_ij <- (a_kk a_ij - a_ik a_kj) / a_{k-1,k-1} is an exact
    division (Sylvester's identity); ``zx.exact_div`` raises if it is not.
    A zero pivot is replaced by the first row below with a non-zero entry in
    that column (one sign flip per exchange); a zero column gives det = 0.
    """
    r = len(M)
    if r == 0:
        return [1]
    A = [[zx.trim(e) for e in row] for row in M]
    sign = 1
    prev = [1]
    for k in range(r - 1):
        if not A[k][k]:
            piv = next((i for i in range(k + 1, r) if A[i][k]), None)
            if piv is None:
                return []
            A[k], A[piv] = A[piv], A[k]
            sign = -sign
        akk = A[k][k]
        for i in range(k + 1, r):
            aik = A[i][k]
            row = A[i]
            for j in range(k + 1, r):
                t = zx.mul(akk, row[j])
                if aik and A[k][j]:
                    t = zx.sub(t, zx.mul(aik, A[k][j]))
                row[j] = zx.exact_div(t, prev) if t else []
            row[k] = []
        prev = akk
    return zx.scale(A[r - 1][r - 1], sign)


def det_int(M):
    """Integer determinant by Bareiss elimination (used for spot values R(a))."""
    r = len(M)
    if r == 0:
        return 1
    A = [list(row) for row in M]
    sign = 1
    prev = 1
    for k in range(r - 1):
        if A[k][k] == 0:
            piv = next((i for i in range(k + 1, r) if A[i][k]), None)
            if piv is None:
                return 0
            A[k], A[piv] = A[piv], A[k]
            sign = -sign
        akk = A[k][k]
        for i in range(k + 1, r):
            aik = A[i][k]
            row = A[i]
            for j in range(k + 1, r):
                q, rem = divmod(akk * row[j] - aik * A[k][j], prev)
                if rem:
                    raise ArithmeticError("Bareiss division not exact")
                row[j] = q
        prev = akk
    return sign * A[r - 1][r - 1]


def det_mod(M, q):
    """Determinant modulo a prime q by Gaussian elimination over F_q."""
    r = len(M)
    A = [[v % q for v in row] for row in M]
    d = 1
    for k in range(r):
        piv = next((i for i in range(k, r) if A[i][k]), None)
        if piv is None:
            return 0
        if piv != k:
            A[k], A[piv] = A[piv], A[k]
            d = -d
        d = d * A[k][k] % q
        inv = pow(A[k][k], q - 2, q)
        for i in range(k + 1, r):
            t = A[i][k] * inv % q
            if t:
                rowi, rowk = A[i], A[k]
                for j in range(k, r):
                    rowi[j] = (rowi[j] - t * rowk[j]) % q
    return d % q


# ----------------------------------------------------------------------------
# the three resultant-type objects of the path

def resultant_y(F, G):
    """R^{(y)} = res(f, g; y) in Z[x] as det of the Sylvester matrix (Section 2)."""
    F = bi_trim(F)
    G = bi_trim(G)
    if not F or not G:
        return []
    return det_zx(sylvester(F, G))


def resultant_x(F, G):
    """R^{(x)} = res(f, g; x) in Z[y]: the y-resultant after exchanging x and y."""
    return resultant_y(bi_transpose(F), bi_transpose(G))


def discriminant_y(F):
    """res(f, f_y; y) as used by Project in Section 3.1 (needs m_y >= 1)."""
    F = bi_trim(F)
    if len(F) < 2:
        raise ValueError("res(f, f_y; y) needs deg_y f >= 1")
    return resultant_y(F, bi_diff_y(F))


def resultant_at(F, G, a):
    """R(a) = det S(f(a,y), g(a,y)) for an integer a, keeping the formal degrees m_y, n_y."""
    F = bi_trim(F)
    G = bi_trim(G)
    if not F or not G:
        return 0
    return det_int(sylvester(bi_eval_x(F, a), bi_eval_x(G, a)))


def resultant_at_mod(F, G, a, q):
    """R(a) mod q with the formal degrees m_y, n_y kept (q prime)."""
    F = bi_trim(F)
    G = bi_trim(G)
    if not F or not G:
        return 0
    fa = [zx.evaluate([c % q for c in r], a) % q for r in F]
    ga = [zx.evaluate([c % q for c in r], a) % q for r in G]
    return det_mod(sylvester(fa, ga), q)
