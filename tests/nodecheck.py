"""Full-size parity of a computed resultant against the oracle's stored node values.

A case record (tests/golden/nodes_*.json, written by
tests/golden/make_node_digests.py from the oracle alone) holds, for
R = res(f, g; y) (or res(f, f_y; y)), the digests of R(a) mod q_k at every node
a = 0..D-1 for primes q_1..q_K.  `check(R, rec)` accepts a computed R exactly
when it equals the oracle's R coefficient for coefficient:

* D - 1 is recomputed here from the Sylvester matrix (oracle.bounds), and
  deg R <= D - 1 is required, so the D node values determine R modulo each q_k;
* every coefficient of the oracle's R is at most B = oracle.bounds.coeff_bound
  in size, and max |coef R| is checked directly, with 2 max(B, max|coef R|) < Q
  = prod q_k; two polynomials that agree modulo Q and lie in (-Q/2, Q/2) are equal.
"""

import math

from oracle.bounds import coeff_bound, degree_bound
from tests.golden.make_golden import input_digest
from tests.golden.make_node_digests import build_inputs, load_group, node_digest, operands


def values_mod(R, q, D):
    """R(a) mod q for a = 0..D-1 (Horner's rule modulo q)."""
    Rq = [c % q for c in R]
    out = []
    for a in range(D):
        v = 0
        for c in reversed(Rq):
            v = (v * a + c) % q
        out.append(v)
    return out


def case(group, name):
    for rec in load_group(group)["cases"]:
        if rec["name"] == name:
            return rec
    raise KeyError(name)


def names(group):
    return [rec["name"] for rec in load_group(group)["cases"]]


def inputs(rec):
    """(kind, f, g) as the library takes them (g = None unless kind is res) and
    the oracle's second Sylvester operand (g, or f_y)."""
    kind, F, G2 = build_inputs(rec)
    return kind, F, (G2 if kind == "res" else None), G2


def check(R, rec):
    kind, F, G, G2 = inputs(rec)
    assert input_digest(F, G) == rec["inputs_sha256"], "inputs changed since the digests were written"
    A, B = operands(kind, F, G2)
    D = degree_bound(A, B) + 1
    assert D == rec["D"], (D, rec["D"])
    assert len(R) <= D, "degree %d above the bound %d" % (len(R) - 1, D - 1)
    primes = [int(q) for q in rec["primes"]]
    Q = math.prod(primes)
    height = max((abs(c) for c in R), default=0)
    assert 2 * max(coeff_bound(A, B), height) < Q, "primes do not fix the result"
    bad = []
    for k, (q, dg) in enumerate(zip(primes, rec["digests"])):
        vals = values_mod(R, q, D)
        if node_digest(vals) != dg:
            bad.append(k)
            if k == 0:
                for a, v in rec["samples_prime0"]:
                    assert vals[a] == int(v), "R(%d) mod q_0 differs from the oracle's" % a
    assert not bad, "node values differ from the oracle's modulo primes %s" % bad
