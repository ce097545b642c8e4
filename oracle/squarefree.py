"""Square-free decomposition in Z[x].  (Test infrastructure; see oracle/__init__.py.)

The curve analysis follows the resultant with its square-free factorisation:
the projection step of Section 3 splits R into square-free parts before
isolating its roots.  The object has a plain definition: for r in Z[x],
r = u * a_1 * a_2^2 * ... * a_k^k with u the signed content of r and the a_i
primitive, square-free, pairwise coprime, positive leading coefficient
(a_i = 1 where r has no factor of multiplicity i), a_k non-constant.

``squarefree_yun`` computes it by Yun's algorithm, each step a gcd in Z[x]
(``oracle.gcd.gcd_zx``) and exact divisions (``oracle.zx.exact_div``):
p = r / u, g = gcd(p, p'), b_1 = p / g, d_1 = p' / g - b_1'; then
a_i = gcd(b_i, d_i), b_{i+1} = b_i / a_i, d_{i+1} = d_i / a_i - b_{i+1}',
until b is constant.  Its pins are planted factorisations and the defining
properties (tests/test_oracle_squarefree.py).
"""

from . import zx
from .gcd import gcd_zx


def derivative(a):
    return zx.trim([i * a[i] for i in range(1, len(a))])


def squarefree_yun(r):
    """(u, [a_1, ..., a_k]) with r = u * prod a_i^i as in the module docstring."""
    r = zx.trim(r)
    if not r:
        return 0, []
    if len(r) == 1:
        return r[0], []
    u = zx.content(r)
    if r[-1] < 0:
        u = -u
    p = [c // u for c in r]
    dp = derivative(p)
    g = gcd_zx(p, dp)
    b = zx.exact_div(p, g)
    d = zx.sub(zx.exact_div(dp, g), derivative(b))
    factors = []
    while len(b) >= 2:
        a = gcd_zx(b, d)
        factors.append(a)
        b2 = zx.exact_div(b, a)
        d = zx.sub(zx.exact_div(d, a), derivative(b2)) if d else []
        b = b2
    return u, factors


def expand(u, factors):
    """u * prod_i factors[i]^(i+1)."""
    out = [u]
    for i, a in enumerate(factors):
        for _ in range(i + 1):
            out = zx.mul(out, a)
    return zx.trim(out)
