"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws random numbers and lays them out; it holds none of the
resultant/gcd arithmetic.  Every generator takes an explicit seed and uses
``numpy.random.Generator(PCG64(seed))``; values wider than 62 bits are built
from 32-bit draws.

Bivariate polynomials are lists of rows: ``F[j][i]`` is the coefficient of
x^i y^j.  "Dense of total degree d" means every coefficient with i + j <= d is
drawn (so the top row j = d is the constant x^0 y^d term).

The workloads stand in for the random dense curves of the paper's experiments
(Section 6, Table 2: dense random curves of given degree and coefficient bit
length); the paper's own instance files are not available.
"""

import math

import numpy as np


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def signed_bits(rng, bits, size):
    """`size` integers uniform in [-2^(bits-1), 2^(bits-1) - 1] (Python ints)."""
    if bits <= 62:
        lo = -(1 << (bits - 1))
        hi = 1 << (bits - 1)
        return [int(v) for v in rng.integers(lo, hi, size=size, dtype=np.int64)]
    words = (bits + 31) // 32
    raw = rng.integers(0, 1 << 32, size=(size, words), dtype=np.uint64)
    mask = (1 << bits) - 1
    half = 1 << (bits - 1)
    out = []
    for row in raw:
        v = 0
        for w in reversed(row):
            v = (v << 32) | int(w)
        out.append((v & mask) - half)
    return out


def inclusive_range(rng, lo, hi, size):
    """`size` integers uniform in [lo, hi] inclusive."""
    return [int(v) for v in rng.integers(lo, hi + 1, size=size, dtype=np.int64)]


def dense_bivariate(rng, tdeg, draw):
    """Dense total-degree-`tdeg` polynomial; `draw(n)` returns n coefficients."""
    F = []
    for j in range(tdeg + 1):
        F.append(draw(tdeg - j + 1))
    return F


def dense_signed(rng, tdeg, bits):
    return dense_bivariate(rng, tdeg, lambda n: signed_bits(rng, bits, n))


def _bimul(F, G):
    """Schoolbook product of two row lists (input construction only)."""
    out = {}
    for j, a in enumerate(F):
        for i, c in enumerate(a):
            if not c:
                continue
            for k, b in enumerate(G):
                for l, d in enumerate(b):
                    if d:
                        out[(j + k, i + l)] = out.get((j + k, i + l), 0) + c * d
    ny = max((j for j, _ in out), default=-1) + 1
    rows = []
    for j in range(ny):
        nx = max((i for (jj, i) in out if jj == j), default=-1) + 1
        rows.append([out.get((j, i), 0) for i in range(nx)])
    return rows


def _biadd(F, G):
    n = max(len(F), len(G))
    rows = []
    for j in range(n):
        a = F[j] if j < len(F) else []
        b = G[j] if j < len(G) else []
        m = max(len(a), len(b))
        rows.append([(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(m)])
    return rows


# ----------------------------------------------------------------------------
# the five workloads (seed = workload index * 1000 + instance)

def pair_deg6(instance=0):
    """Dense total degree 6, coefficients uniform in [-2^10, 2^10]."""
    rng = rng_for(1000 + instance)
    draw = lambda n: inclusive_range(rng, -(1 << 10), 1 << 10, n)
    return dense_bivariate(rng, 6, draw), dense_bivariate(rng, 6, draw)


def pair_deg20(instance=0):
    """Dense total degree 20, uniform 32-bit signed coefficients."""
    rng = rng_for(2000 + instance)
    return dense_signed(rng, 20, 32), dense_signed(rng, 20, 32)


def curve_deg40(instance=0, tdeg=40, bits=16):
    """Curve for res(f, f_y; y): dense total degree 40, 16-bit signed coefficients."""
    rng = rng_for(3000 + instance)
    return dense_signed(rng, tdeg, bits)


def singular_curve_deg40(instance=0, dg=20, dh=20, dk=20, bits=8, square_k=False):
    """f = g^2 + h*k (or g^2 + h*k^2 with square_k) from dense g, h, k."""
    rng = rng_for(3500 + instance)
    g = dense_signed(rng, dg, bits)
    h = dense_signed(rng, dh, bits)
    k = dense_signed(rng, dk, bits)
    hk = _bimul(h, _bimul(k, k) if square_k else k)
    return _biadd(_bimul(g, g), hk)


def arrangement_batch(instance=0, n_curves=400, group=20, deg_range=(4, 30), bits_range=(8, 64)):
    """400 curves (total degree U{4..30}, bits U{8..64}); all pairs inside
    seeded groups of 20.  Returns (curves, pairs) with pairs as index tuples."""
    rng = rng_for(4000 + instance)
    degs = inclusive_range(rng, deg_range[0], deg_range[1], n_curves)
    bits = inclusive_range(rng, bits_range[0], bits_range[1], n_curves)
    curves = [dense_signed(rng, d, b) for d, b in zip(degs, bits)]
    perm = [int(v) for v in rng.permutation(n_curves)]
    pairs = []
    for g0 in range(0, n_curves, group):
        members = perm[g0:g0 + group]
        for a in range(len(members)):
            for b in range(a + 1, len(members)):
                pairs.append((members[a], members[b]))
    return curves, pairs


def poisson_requests(instance=0, n=2000, qps=100.0, deg_range=(5, 64), bits_range=(10, 128), p_disc=0.5):
    """Poisson arrivals.  Each request: kind ('res' or 'disc'), shared total
    degree round(exp(U[ln 5, ln 64])), coefficient bits U{10..128}, f and g."""
    rng = rng_for(5000 + instance)
    gaps = rng.exponential(1.0 / qps, size=n)
    t = 0.0
    reqs = []
    for r in range(n):
        t += float(gaps[r])
        kind = "disc" if rng.random() < p_disc else "res"
        d = int(round(math.exp(rng.uniform(math.log(deg_range[0]), math.log(deg_range[1])))))
        b = inclusive_range(rng, bits_range[0], bits_range[1], 1)[0]
        f = dense_signed(rng, d, b)
        g = dense_signed(rng, d, b) if kind == "res" else None
        reqs.append({"t": t, "kind": kind, "tdeg": d, "bits": b, "f": f, "g": g})
    return reqs


def random_dense(seed, tdeg, bits):
    """Generic dense pair for parity sweeps."""
    rng = rng_for(seed)
    return dense_signed(rng, tdeg, bits), dense_signed(rng, tdeg, bits)


def random_rect(seed, ydeg_f, xdeg_f, ydeg_g, xdeg_g, bits, zero_frac=0.0):
    """Pair with rectangular supports (y-degree, x-degree per row) and optional sparsity."""
    rng = rng_for(seed)

    def one(ny, nx):
        rows = []
        for j in range(ny + 1):
            row = signed_bits(rng, bits, nx + 1)
            if zero_frac > 0:
                mask = rng.random(nx + 1) < zero_frac
                row = [0 if z else v for v, z in zip(row, mask)]
            rows.append(row)
        return rows

    return one(ydeg_f, xdeg_f), one(ydeg_g, xdeg_g)
