"""Dense univariate polynomials over Z.  (Test infrastructure; see oracle/__init__.py.)

A polynomial is a Python list of ints in ascending powers, ``a[i]`` being the
coefficient of x^i.  The zero polynomial is ``[]``; every function returns
trimmed lists (no trailing zero coefficients).

Multiplication packs each polynomial into one integer (Kronecker substitution
x -> 2^b with a b wide enough for every product coefficient, signed digits), so
that CPython's big-integer product does the work; exact division packs the same
way and divides the integers, which is exact whenever the polynomial division
is.  Both are library primitives used as single steps.
"""

from math import gcd as _igcd


def trim(a):
    """Drop trailing zero coefficients; [] is the zero polynomial."""
    n = len(a)
    while n and a[n - 1] == 0:
        n -= 1
    return list(a[:n])


def deg(a):
    """Degree of a trimmed or untrimmed polynomial; -1 for zero."""
    return len(trim(a)) - 1


def add(a, b):
    n = max(len(a), len(b))
    return trim([(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)])


def neg(a):
    return [-c for c in trim(a)]


def sub(a, b):
    return add(a, neg(b))


def scale(a, c):
    return trim([c * v for v in a])


def height(a):
    """Max |coefficient| (0 for the zero polynomial)."""
    return max((abs(c) for c in a), default=0)


def _pack(a, bits):
    v = 0
    for c in reversed(a):
        v = (v << bits) + c
    return v


def _unpack(v, bits, n):
    """Inverse of _pack for n signed digits each of magnitude < 2^(bits-1)."""
    out = []
    mask = (1 << bits) - 1
    half = 1 << (bits - 1)
    for _ in range(n):
        d = v & mask
        if d >= half:
            d -= 1 << bits
        out.append(d)
        v = (v - d) >> bits
    if v != 0:
        raise ArithmeticError("Kronecker unpack overflow")
    return trim(out)


def mul(a, b):
    """Product in Z[x] via Kronecker substitution."""
    a = trim(a)
    b = trim(b)
    if not a or not b:
        return []
    if len(a) == 1:
        return scale(b, a[0])
    if len(b) == 1:
        return scale(a, b[0])
    bound = height(a) * height(b) * min(len(a), len(b))
    bits = bound.bit_length() + 2
    return _unpack(_pack(a, bits) * _pack(b, bits), bits, len(a) + len(b) - 1)


def exact_div(n, d):
    """Quotient q with n = q*d in Z[x]; raises if the division is not exact.

    The quotient's coefficients obey the Landau-Mignotte factor bound
    |q_i| <= 2^deg(q) * ||n||_2, so packing with that many bits recovers q.
    """
    n = trim(n)
    d = trim(d)
    if not d:
        raise ZeroDivisionError("division by the zero polynomial")
    if not n:
        return []
    if len(d) == 1:
        q = []
        for c in n:
            qq, r = divmod(c, d[0])
            if r:
                raise ArithmeticError("inexact division by a constant")
            q.append(qq)
        return trim(q)
    dq = len(n) - len(d)
    if dq < 0:
        raise ArithmeticError("inexact division (degree)")
    bits = height(n).bit_length() + dq + (len(n).bit_length() + 1) // 2 + 3
    nv = _pack(n, bits)
    dv = _pack(d, bits)
    qv, r = divmod(nv, dv)
    if r:
        raise ArithmeticError("inexact polynomial division")
    q = _unpack(qv, bits, dq + 1)
    if len(q) != dq + 1:
        raise ArithmeticError("inexact polynomial division (quotient degree)")
    return q


def divmod_q(n, d):
    """Quotient and remainder over Q (lists of fractions.Fraction)."""
    from fractions import Fraction
    n = [Fraction(c) for c in trim(n)]
    d = [Fraction(c) for c in trim(d)]
    if not d:
        raise ZeroDivisionError
    q = [Fraction(0)] * max(len(n) - len(d) + 1, 0)
    r = list(n)
    while len(r) >= len(d) and r:
        s = len(r) - len(d)
        t = r[-1] / d[-1]
        q[s] = t
        for i, c in enumerate(d):
            r[s + i] -= t * c
        while r and r[-1] == 0:
            r.pop()
    return q, r


def evaluate(a, x):
    """a(x) for an integer (or Fraction) x, by Horner's rule."""
    v = 0
    for c in reversed(trim(a)):
        v = v * x + c
    return v


def derivative(a):
    return trim([i * a[i] for i in range(1, len(a))])


def power(a, e):
    r = [1]
    for _ in range(e):
        r = mul(r, a)
    return r


def content(a):
    """gcd of the coefficients (non-negative; 0 for the zero polynomial)."""
    c = 0
    for v in trim(a):
        c = _igcd(c, v)
    return c


def primitive_part(a):
    a = trim(a)
    if not a:
        return []
    c = content(a)
    if a[-1] < 0:
        c = -c
    return [v // c for v in a]
