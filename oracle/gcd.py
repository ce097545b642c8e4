"""gcd in Z[x] and in F_p[x].  (Test infrastructure; see oracle/__init__.py.)

Section 5.1 ("Computing gcds in Z[x]") computes gcd(f, g) for f, g in Z[x] by
Brown's modular method.  The object it reconstructs has this plain definition,
which is what ``gcd_zx`` computes: the gcd over Q, scaled to a primitive
integer polynomial with positive leading coefficient, times the gcd of the two
contents.  ``gcd_zx`` runs the primitive remainder sequence over Z;
``gcd_q_euclid`` runs Euclid over Q directly and pins it on small inputs.

Normalisation (the paper leaves it open): gcd(0, 0) = 0 (the empty list);
gcd(a, 0) = a with positive leading coefficient.
"""

from fractions import Fraction
from math import gcd as _igcd, lcm as _ilcm

from . import zx


def _normalise_sign(a):
    a = zx.trim(a)
    if a and a[-1] < 0:
        a = [-c for c in a]
    return a


def prem(u, v):
    """Pseudo-remainder: lc(v)^(deg u - deg v + 1) u mod v, computed over Z."""
    u = zx.trim(u)
    v = zx.trim(v)
    lv = v[-1]
    e = len(u) - len(v) + 1
    r = list(u)
    while len(r) >= len(v) and r:
        s = len(r) - len(v)
        t = r[-1]
        r = [lv * c for c in r]
        for i, c in enumerate(v):
            r[s + i] -= t * c
        e -= 1
        r = zx.trim(r)
    return [c * lv ** e for c in r] if e > 0 else r


def gcd_zx(a, b):
    """gcd in Z[x]: gcd of the contents times the primitive gcd, positive lc.

    The primitive gcd is the last non-zero term of the primitive remainder
    sequence u, v, pp(prem(u, v)), ... started from the primitive parts; each
    pseudo-remainder is an associate over Q of the Euclidean remainder, so the
    sequence ends at an associate of the gcd over Q (Euclid's algorithm over Q
    with the denominators cleared).
    """
    a = zx.trim(a)
    b = zx.trim(b)
    if not a and not b:
        return []
    if not b:
        return _normalise_sign(a)
    if not a:
        return _normalise_sign(b)
    c = _igcd(zx.content(a), zx.content(b))
    u, v = zx.primitive_part(a), zx.primitive_part(b)
    if len(u) < len(v):
        u, v = v, u
    while v:
        r = prem(u, v)
        u, v = v, zx.primitive_part(r) if r else []
    return [c * t for t in zx.primitive_part(u)]


def gcd_q_euclid(a, b):
    """The same gcd by Euclid's algorithm over Q (Fractions); slow, small inputs only."""
    a = zx.trim(a)
    b = zx.trim(b)
    if not a and not b:
        return []
    if not b:
        return _normalise_sign(a)
    if not a:
        return _normalise_sign(b)
    c = _igcd(zx.content(a), zx.content(b))
    u = [Fraction(v) for v in a]
    v = [Fraction(w) for w in b]
    while v:
        _, r = zx.divmod_q(u, v)
        u, v = v, r
    den = 1
    for t in u:
        den = _ilcm(den, t.denominator)
    h = zx.primitive_part([int(t * den) for t in u])
    return [c * t for t in h]


def gcd_mod_p(a, b, p):
    """Monic gcd over F_p (p prime) by Euclid; [] if both are zero mod p."""
    def tr(v):
        v = [x % p for x in v]
        while v and v[-1] == 0:
            v.pop()
        return v

    u, v = tr(a), tr(b)
    while v:
        inv = pow(v[-1], p - 2, p)
        r = list(u)
        while len(r) >= len(v):
            s = len(r) - len(v)
            t = r[-1] * inv % p
            for i, c in enumerate(v):
                r[s + i] = (r[s + i] - t * c) % p
            r = tr(r)
        u, v = v, r
    if not u:
        return []
    inv = pow(u[-1], p - 2, p)
    return [x * inv % p for x in u]
