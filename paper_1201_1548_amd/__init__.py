"""Exact bivariate resultants, discriminants and gcds on MI355X (gfx950).

Python binding of the C ABI in include/bires.h: argument marshalling only.
Every step of the computation runs in the HIP kernels of libbires.so; there is
no CPU fallback, and a missing library raises at the first call.

Bivariate polynomials are lists of rows, ``F[j][i]`` the coefficient of
x^i y^j (Python ints of any size); univariate results are lists of ints in
ascending powers of x, ``[]`` for the zero polynomial.
"""

import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))

VAR_X, VAR_Y = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
KIND_RESULTANT, KIND_DISCRIMINANT, KIND_POLAR = 0, 1, 2
_KINDS = {"res": KIND_RESULTANT, "disc": KIND_DISCRIMINANT, "polar": KIND_POLAR}

ERRORS = {
    -1: "EINVAL", -2: "EBUFSIZE", -3: "ENOMEM", -4: "ETOOBIG",
    -5: "EDEVICE", -6: "ECHECK", -7: "ENOTFOUND", -8: "ETIMEOUT",
}
E_BUFSIZE = -2


class BiresError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (what, ERRORS.get(code, "?"), code))


class Bipoly(ctypes.Structure):
    _fields_ = [("deg_y", ctypes.c_int32), ("deg_x", ctypes.c_int32), ("limbs", ctypes.c_int32),
                ("c", ctypes.c_void_p)]


class Upoly(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("limbs", ctypes.c_int32), ("c", ctypes.c_void_p)]


_lib = None

_SIGS = {
    "bires_init": ([], ctypes.c_int),
    "bires_resultant_bounds": ([ctypes.POINTER(Bipoly), ctypes.POINTER(Bipoly), ctypes.c_int,
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "bires_resultant": ([ctypes.POINTER(Bipoly), ctypes.POINTER(Bipoly), ctypes.c_int, ctypes.POINTER(Upoly),
                         ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "bires_discriminant_bounds": ([ctypes.POINTER(Bipoly), ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "bires_discriminant": ([ctypes.POINTER(Bipoly), ctypes.c_int, ctypes.POINTER(Upoly), ctypes.c_int,
                            ctypes.c_void_p], ctypes.c_int),
    "bires_polar_bounds": ([ctypes.POINTER(Bipoly), ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                            ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "bires_polar_resultant": ([ctypes.POINTER(Bipoly), ctypes.c_int, ctypes.POINTER(Upoly), ctypes.c_int,
                               ctypes.c_void_p], ctypes.c_int),
    "bires_psc": ([ctypes.POINTER(Bipoly), ctypes.POINTER(Bipoly), ctypes.c_int, ctypes.c_int, ctypes.c_uint32,
                   ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                   ctypes.c_void_p], ctypes.c_int),
    "bires_fiber_bounds": ([ctypes.POINTER(Bipoly), ctypes.c_int, ctypes.POINTER(Upoly), ctypes.c_int32,
                            ctypes.c_uint32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                            ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p], ctypes.c_int),
    "bires_gcd_bounds": ([ctypes.POINTER(Upoly), ctypes.POINTER(Upoly), ctypes.POINTER(ctypes.c_int32),
                          ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "bires_gcd": ([ctypes.POINTER(Upoly), ctypes.POINTER(Upoly), ctypes.POINTER(Upoly), ctypes.c_int,
                   ctypes.c_void_p], ctypes.c_int),
    "bires_squarefree": ([ctypes.POINTER(Upoly), ctypes.POINTER(Upoly), ctypes.POINTER(Upoly), ctypes.c_int32,
                          ctypes.POINTER(ctypes.c_int32), ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "bires_resultant_noalloc": ([ctypes.POINTER(Bipoly), ctypes.POINTER(Bipoly), ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(Upoly), ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "bires_resultant_batch": ([ctypes.c_int, ctypes.POINTER(Bipoly), ctypes.POINTER(Bipoly),
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(Upoly), ctypes.POINTER(ctypes.c_int32), ctypes.c_int,
                               ctypes.c_void_p], ctypes.c_int),
    "bires_resultant_batch_async": ([ctypes.c_int, ctypes.POINTER(Bipoly), ctypes.POINTER(Bipoly),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(Upoly), ctypes.POINTER(ctypes.c_int32), ctypes.c_int,
                                     ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "bires_batch_wait": ([ctypes.c_uint64], ctypes.c_int),
    "bires_server_create": ([ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "bires_server_submit": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Bipoly),
                             ctypes.POINTER(Bipoly), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "bires_server_wait": ([ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Upoly), ctypes.c_double,
                           ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "bires_server_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "bires_plan": ([ctypes.POINTER(Bipoly), ctypes.POINTER(Bipoly), ctypes.c_int, ctypes.c_int,
                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                    ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "bires_primes": ([ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "bires_debug_values": ([ctypes.POINTER(Bipoly), ctypes.POINTER(Bipoly), ctypes.c_int, ctypes.c_int,
                            ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                            ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "bires_set_timing": ([ctypes.c_int], ctypes.c_int),
    "bires_set_schedule": ([ctypes.c_int], ctypes.c_int),
    "bires_set_graphs": ([ctypes.c_int], ctypes.c_int),
    "bires_set_eval_kernel": ([ctypes.c_int], ctypes.c_int),
    "bires_set_plan_cache": ([ctypes.c_int], ctypes.c_int),
    "bires_issue_rates": ([ctypes.POINTER(ctypes.c_double), ctypes.c_int], ctypes.c_int),
    "bires_plan_cache_stats": ([ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "bires_schur_stats": ([ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "bires_graph_stats": ([ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "bires_autotune": ([ctypes.c_int, ctypes.POINTER(Bipoly), ctypes.POINTER(Bipoly),
                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Upoly),
                        ctypes.POINTER(ctypes.c_int32), ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                        ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "bires_kernel_time": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "bires_host_time": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "bires_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "bires_device_info": ([ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
}


def lib():
    """The loaded libbires.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            raise RuntimeError("libbires.so is not built (run __graft_entry__.build() or "
                               "python -m paper_1201_1548_amd.build); there is no fallback path")
        # One HIP runtime per process: torch ships its own libamdhip64 (soname
        # libamdhip64.so.7).  Loading torch first makes the dynamic loader bind
        # libbires to that same runtime, so torch's streams and device pointers
        # are valid in the library.  (Importing torch does not touch the GPU.)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(path)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(code, what):
    if code != 0:
        raise BiresError(code, what)


# ----------------------------------------------------------------------------
# marshalling of integers <-> two's-complement 32-bit limbs

def limbs_needed(values):
    bits = 1
    for v in values:
        b = (v if v >= 0 else ~v).bit_length() + 1
        if b > bits:
            bits = b
    return (bits + 31) // 32


def ints_to_limbs(values, L):
    """Python ints -> uint32 array [len(values), L] (two's complement)."""
    n = len(values)
    if L == 1:
        return np.array([v & 0xFFFFFFFF for v in values], dtype=np.uint32).reshape(n, 1)
    nb = 4 * L
    buf = b"".join(v.to_bytes(nb, "little", signed=True) for v in values)
    return np.frombuffer(buf, dtype="<u4").reshape(n, L).copy()


def limbs_to_ints(arr):
    """uint32 array [n, L] -> Python ints (two's complement)."""
    n, L = arr.shape
    raw = np.ascontiguousarray(arr, dtype="<u4").tobytes()
    nb = 4 * L
    return [int.from_bytes(raw[r * nb:(r + 1) * nb], "little", signed=True) for r in range(n)]


def bipoly_array(F, limbs=None):
    """Rows F[j][i] -> uint32 array [rows, cols, L] (dense rectangle)."""
    rows = len(F)
    cols = max((len(r) for r in F), default=0)
    flat = [F[j][i] if i < len(F[j]) else 0 for j in range(rows) for i in range(cols)]
    L = limbs or limbs_needed(flat)
    arr = ints_to_limbs(flat, L).reshape(rows, cols, L)
    return arr


def _desc(arr, ptr=None):
    rows, cols, L = arr.shape
    d = Bipoly()
    d.deg_y = rows - 1 if rows * cols else -1
    d.deg_x = cols - 1 if rows * cols else -1
    d.limbs = L
    d.c = ptr if ptr is not None else arr.ctypes.data
    return d


class DeviceBipoly:
    """A bivariate input resident in device memory (a torch uint32-word tensor)."""

    def __init__(self, F, limbs=None, device="cuda"):
        import torch
        arr = bipoly_array(F, limbs)
        self.shape = arr.shape
        self.tensor = torch.from_numpy(arr.view(np.int32)).to(device)

    def desc(self):
        rows, cols, L = self.shape
        d = Bipoly()
        d.deg_y = rows - 1 if rows * cols else -1
        d.deg_x = cols - 1 if rows * cols else -1
        d.limbs = L
        d.c = self.tensor.data_ptr()
        return d


def _bounds(kind, fd, gd, var):
    deg = ctypes.c_int32()
    L = ctypes.c_int32()
    if kind == KIND_RESULTANT:
        _check(lib().bires_resultant_bounds(ctypes.byref(fd), ctypes.byref(gd), var, ctypes.byref(deg),
                                            ctypes.byref(L)), "bires_resultant_bounds")
    elif kind == KIND_DISCRIMINANT:
        _check(lib().bires_discriminant_bounds(ctypes.byref(fd), var, ctypes.byref(deg), ctypes.byref(L)),
               "bires_discriminant_bounds")
    else:
        _check(lib().bires_polar_bounds(ctypes.byref(fd), var, ctypes.byref(deg), ctypes.byref(L)),
               "bires_polar_bounds")
    return deg.value, L.value


def _kind(kind):
    """Job kind code of 'res', 'disc' (res(f, df/dvar)) or 'polar' (res(df/dother, df/dvar))."""
    if kind in _KINDS.values():
        return kind
    if kind not in _KINDS:
        raise ValueError("kind must be 'res', 'disc' or 'polar'")
    return _KINDS[kind]


def _var(var):
    if var in ("x", VAR_X):
        return VAR_X
    if var in ("y", VAR_Y):
        return VAR_Y
    raise ValueError("var must be 'x' or 'y'")


def _stream(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(stream)


def resultant(F, G, var="y", stream=None):
    """res(f, g; var) as a list of Python ints (host-memory call)."""
    v = _var(var)
    fa, ga = bipoly_array(F), bipoly_array(G)
    fd, gd = _desc(fa), _desc(ga)
    deg, L = _bounds(KIND_RESULTANT, fd, gd, v)
    out = np.zeros((deg + 1, L), dtype=np.uint32)
    od = Upoly(deg, L, out.ctypes.data)
    _check(lib().bires_resultant(ctypes.byref(fd), ctypes.byref(gd), v, ctypes.byref(od), MEM_HOST,
                                 _stream(stream)), "bires_resultant")
    return limbs_to_ints(out[: od.degree + 1])


def discriminant(F, var="y", stream=None):
    """res(f, df/dvar; var) as a list of Python ints (host-memory call)."""
    v = _var(var)
    fa = bipoly_array(F)
    fd = _desc(fa)
    deg, L = _bounds(KIND_DISCRIMINANT, fd, fd, v)
    out = np.zeros((deg + 1, L), dtype=np.uint32)
    od = Upoly(deg, L, out.ctypes.data)
    _check(lib().bires_discriminant(ctypes.byref(fd), v, ctypes.byref(od), MEM_HOST, _stream(stream)),
           "bires_discriminant")
    return limbs_to_ints(out[: od.degree + 1])


def polar_resultant(F, var="y", stream=None):
    """res(df/dother, df/dvar; var) -- for var 'y' the Q = res(f_x, f_y; y) of the
    fiber bound n_alpha^+ (generic case gcd(f_x, f_y) = 1) -- as a list of
    Python ints (host-memory call)."""
    v = _var(var)
    fa = bipoly_array(F)
    fd = _desc(fa)
    deg, L = _bounds(KIND_POLAR, fd, fd, v)
    out = np.zeros((deg + 1, L), dtype=np.uint32)
    od = Upoly(deg, L, out.ctypes.data)
    _check(lib().bires_polar_resultant(ctypes.byref(fd), v, ctypes.byref(od), MEM_HOST, _stream(stream)),
           "bires_polar_resultant")
    return limbs_to_ints(out[: od.degree + 1])


def resultant_noalloc(F, G=None, kind="res", var="y", stream=None, device=False):
    """res(f, g; var) (kind "res"), res(f, df/dvar; var) (kind "disc") or
    res(df/dother, df/dvar; var) (kind "polar") through
    the allocation-free entry point bires_resultant_noalloc.  device=True
    passes device-memory inputs and output (torch tensors), else host memory.
    The library must be set up first (init())."""
    k = _kind(kind)
    v = _var(var)
    fa = bipoly_array(F)
    ga = bipoly_array(G) if k == KIND_RESULTANT else fa
    fd, gd = _desc(fa), _desc(ga)
    deg, L = _bounds(k, fd, gd, v)
    if not device:
        out = np.zeros((deg + 1, L), dtype=np.uint32)
        od = Upoly(deg, L, out.ctypes.data)
        _check(lib().bires_resultant_noalloc(ctypes.byref(fd), ctypes.byref(gd), k, v, ctypes.byref(od), MEM_HOST,
                                             _stream(stream)), "bires_resultant_noalloc")
        return limbs_to_ints(out[: od.degree + 1])
    import torch
    tf = torch.from_numpy(fa.view(np.int32)).cuda()
    tg = torch.from_numpy(ga.view(np.int32)).cuda()
    tout = torch.zeros((deg + 1, L), dtype=torch.int32, device="cuda")
    fd, gd = _desc(fa, tf.data_ptr()), _desc(ga, tg.data_ptr())
    od = Upoly(deg, L, tout.data_ptr())
    torch.cuda.synchronize()
    _check(lib().bires_resultant_noalloc(ctypes.byref(fd), ctypes.byref(gd), k, v, ctypes.byref(od), MEM_DEVICE,
                                         _stream(stream)), "bires_resultant_noalloc")
    return limbs_to_ints(tout.cpu().numpy().view(np.uint32)[: od.degree + 1])


def psc(F, G=None, kind="res", var="y", prime=None, stream=None):
    """Principal subresultant coefficients modulo one library prime
    (bires_psc): returns (p, [sr_0 mod p, sr_1 mod p, ...]), each a trimmed list
    of ints in [0, p) in ascending powers of the other variable.  prime: a
    library prime (default: the first, primes(1)[0])."""
    k = _kind(kind)
    p = primes(1)[0] if prime is None else int(prime)
    fa = bipoly_array(F)
    ga = bipoly_array(G) if k == KIND_RESULTANT else fa
    fd, gd = _desc(fa), _desc(ga)
    count = ctypes.c_int32()
    pts = ctypes.c_int32()
    code = lib().bires_psc(ctypes.byref(fd), ctypes.byref(gd), k, _var(var), p, None, 0, ctypes.byref(count),
                           ctypes.byref(pts), _stream(stream))
    if code != E_BUFSIZE and code != 0:
        _check(code, "bires_psc")
    n = count.value * pts.value
    out = np.zeros(max(n, 1), dtype=np.uint32)
    if n:
        _check(lib().bires_psc(ctypes.byref(fd), ctypes.byref(gd), k, _var(var), p, out.ctypes.data, n,
                               ctypes.byref(count), ctypes.byref(pts), _stream(stream)), "bires_psc")
    rows = []
    for i in range(count.value):
        r = [int(v) for v in out[i * pts.value:(i + 1) * pts.value]]
        while r and r[-1] == 0:
            r.pop()
        rows.append(r)
    return p, rows


def fiber_bounds(F, rstar, deg_r, var="y", prime=None, stream=None):
    """(N^-, N^+, flags) of the modular generic-position test (bires_fiber_bounds)
    for the curve F, the square-free part rstar of R = res(f, f_y; y) and deg R."""
    p = primes(1)[0] if prime is None else int(prime)
    fa = bipoly_array(F)
    fd = _desc(fa)
    ra, rd = _upoly_in(rstar)
    nm = ctypes.c_int64()
    npl = ctypes.c_int64()
    fl = ctypes.c_int32()
    _check(lib().bires_fiber_bounds(ctypes.byref(fd), _var(var), ctypes.byref(rd), int(deg_r), p, ctypes.byref(nm),
                                    ctypes.byref(npl), ctypes.byref(fl), _stream(stream)), "bires_fiber_bounds")
    return nm.value, npl.value, fl.value


def init():
    """Set up the library on the current device (bires_init)."""
    _check(lib().bires_init(), "bires_init")


def _upoly_in(a):
    a = list(a)
    while a and a[-1] == 0:
        a.pop()
    L = limbs_needed(a) if a else 1
    arr = ints_to_limbs(a, L) if a else np.zeros((1, 1), dtype=np.uint32)
    return arr, Upoly(len(a) - 1, L, arr.ctypes.data)


def gcd(a, b, stream=None):
    """gcd(a, b) in Z[x] (host-memory call)."""
    aa, ad = _upoly_in(a)
    ba, bd = _upoly_in(b)
    deg = ctypes.c_int32()
    L = ctypes.c_int32()
    _check(lib().bires_gcd_bounds(ctypes.byref(ad), ctypes.byref(bd), ctypes.byref(deg), ctypes.byref(L)),
           "bires_gcd_bounds")
    out = np.zeros((max(deg.value, 0) + 1, L.value), dtype=np.uint32)
    od = Upoly(max(deg.value, 0), L.value, out.ctypes.data)
    _check(lib().bires_gcd(ctypes.byref(ad), ctypes.byref(bd), ctypes.byref(od), MEM_HOST, _stream(stream)),
           "bires_gcd")
    return limbs_to_ints(out[: od.degree + 1])


def squarefree(r, stream=None):
    """Square-free decomposition (bires_squarefree): returns (u, [a_1, ..., a_k])
    with r = u * a_1 * a_2^2 * ... * a_k^k (host-memory call; the output sizes
    are grown and the call repeated when the library reports them too small)."""
    ra, rd = _upoly_in(r)
    deg = max(len(r) - 1, 0)
    cap_deg, cap_L = deg, int(ra.shape[1]) + 2
    nmax = min(max(deg, 1), 8)  # grown when the library reports more factors
    degs, Ls = [cap_deg] * nmax, [cap_L] * nmax
    udeg, uL = 0, cap_L
    for _ in range(4):
        ubuf = np.zeros((udeg + 1, uL), dtype=np.uint32)
        ud = Upoly(udeg, uL, ubuf.ctypes.data)
        bufs = [np.zeros((degs[i] + 1, Ls[i]), dtype=np.uint32) for i in range(nmax)]
        fds = (Upoly * nmax)()
        for i in range(nmax):
            fds[i] = Upoly(degs[i], Ls[i], bufs[i].ctypes.data)
        count = ctypes.c_int32()
        code = lib().bires_squarefree(ctypes.byref(rd), ctypes.byref(ud), fds, nmax, ctypes.byref(count), MEM_HOST,
                                      _stream(stream))
        if code == E_BUFSIZE:
            udeg, uL = max(udeg, ud.degree), max(uL, ud.limbs)
            for i in range(nmax):
                degs[i], Ls[i] = max(degs[i], fds[i].degree), max(Ls[i], fds[i].limbs)
            if count.value > nmax:
                degs += [cap_deg] * (count.value - nmax)
                Ls += [cap_L] * (count.value - nmax)
                nmax = count.value
            continue
        _check(code, "bires_squarefree")
        u = limbs_to_ints(ubuf[: ud.degree + 1]) if ud.degree >= 0 else []
        facs = [limbs_to_ints(bufs[i][: fds[i].degree + 1]) for i in range(count.value)]
        return (u[0] if u else 0), facs
    raise BiresError(E_BUFSIZE, "bires_squarefree: output sizes did not settle")


def resultant_batch(jobs, stream=None):
    """jobs: list of (kind, F, G, var) with kind 'res', 'disc' or 'polar' (G ignored
    unless 'res').
    Returns (results, statuses); one batched launch sequence for all jobs."""
    n = len(jobs)
    keep = []
    fds = (Bipoly * n)()
    gds = (Bipoly * n)()
    kinds = (ctypes.c_int32 * n)()
    vars_ = (ctypes.c_int32 * n)()
    outs = (Upoly * n)()
    bufs = []
    for i, (kind, F, G, var) in enumerate(jobs):
        k = _kind(kind)
        fa = bipoly_array(F)
        ga = bipoly_array(G) if k == KIND_RESULTANT else fa
        keep += [fa, ga]
        fds[i] = _desc(fa)
        gds[i] = _desc(ga)
        kinds[i] = k
        vars_[i] = _var(var)
        try:
            deg, L = _bounds(k, fds[i], gds[i], vars_[i])
        except BiresError:
            deg, L = 0, 1          # the batch call reports this job's error in status
        out = np.zeros((deg + 1, L), dtype=np.uint32)
        bufs.append(out)
        outs[i] = Upoly(deg, L, out.ctypes.data)
    status = (ctypes.c_int32 * n)()
    lib().bires_resultant_batch(n, fds, gds, kinds, vars_, outs, status, MEM_HOST, _stream(stream))
    res = []
    for i in range(n):
        res.append(limbs_to_ints(bufs[i][: outs[i].degree + 1]) if status[i] == 0 else None)
    return res, list(status)


def plan(F, G=None, kind="res", var="y"):
    """(points D, primes P, log2 of the coefficient bound) of a job; host-only."""
    k = _kind(kind)
    fa = bipoly_array(F)
    ga = bipoly_array(G) if G is not None else fa
    fd, gd = _desc(fa), _desc(ga)
    D = ctypes.c_int32()
    P = ctypes.c_int32()
    lb = ctypes.c_double()
    _check(lib().bires_plan(ctypes.byref(fd), ctypes.byref(gd), k, _var(var), ctypes.byref(D), ctypes.byref(P),
                            ctypes.byref(lb)), "bires_plan")
    return D.value, P.value, lb.value


def bounds(F, G=None, kind="res", var="y"):
    """(max degree, max limbs) from the extents of the inputs; host-only."""
    k = _kind(kind)
    fa = bipoly_array(F)
    ga = bipoly_array(G) if G is not None else fa
    return _bounds(k, _desc(fa), _desc(ga), _var(var))


def primes(n):
    out = np.zeros(max(n, 1), dtype=np.uint32)
    _check(lib().bires_primes(n, out.ctypes.data), "bires_primes")
    return [int(v) for v in out[:n]]


def debug_values(F, G=None, kind="res", var="y"):
    """Stage view: (primes, values[P][D]) of the univariate resultants at a = 0..D-1."""
    k = _kind(kind)
    D, P, _ = plan(F, G, kind, var)
    fa = bipoly_array(F)
    ga = bipoly_array(G) if G is not None else fa
    fd, gd = _desc(fa), _desc(ga)
    vals = np.zeros(P * D, dtype=np.uint32)
    Dp = ctypes.c_int32()
    Pp = ctypes.c_int32()
    _check(lib().bires_debug_values(ctypes.byref(fd), ctypes.byref(gd), k, _var(var), vals.ctypes.data,
                                    vals.size, ctypes.byref(Dp), ctypes.byref(Pp)), "bires_debug_values")
    return primes(Pp.value), vals.reshape(Pp.value, Dp.value)


SCHEDULE_STAGED, SCHEDULE_FUSED, SCHEDULE_AUTO, SCHEDULE_SCHUR = 0, 1, 2, 3


def set_schedule(schedule):
    """Launch schedule of batched calls: 'staged', 'fused', 'schur' (staged with
    the Schur elimination, a wavefront per instance) or 'auto'."""
    code = {"staged": 0, "fused": 1, "auto": 2, "schur": 3}[schedule] if isinstance(schedule, str) else schedule
    _check(lib().bires_set_schedule(code), "bires_set_schedule")


def set_eval_kernel(kernel):
    """Evaluation + elimination kernel of the staged schedule: 'auto' (f's
    array in registers where the degrees allow), 'lds' or 'schur' (the Schur
    algorithm on the displacement generators, a wavefront per instance).  The
    fused schedule follows 'auto' and 'lds', and runs the LDS kernel's
    function in place of Schur."""
    _check(lib().bires_set_eval_kernel({"auto": 0, "lds": 1, "schur": 2}[kernel]), "bires_set_eval_kernel")


def schur_stats():
    """(instances run on the Schur kernel, of them recomputed by Euclid) since set-up."""
    a = ctypes.c_int64()
    b = ctypes.c_int64()
    _check(lib().bires_schur_stats(ctypes.byref(a), ctypes.byref(b)), "bires_schur_stats")
    return a.value, b.value


ISSUE_RATE_INSTRUCTIONS = ("v_add_u32", "v_min_u32", "v_mul_lo_u32", "v_mad_u64_u32", "v_fma_f64",
                           "v_mfma_i32_32x32x32_i8")


def issue_rates():
    """SIMD cycles per wave64 instruction of single VALU and matrix-core instructions (dict)."""
    c = (ctypes.c_double * len(ISSUE_RATE_INSTRUCTIONS))()
    _check(lib().bires_issue_rates(c, len(c)), "bires_issue_rates")
    return dict(zip(ISSUE_RATE_INSTRUCTIONS, list(c)))


def set_plan_cache(enable):
    """Reuse of the previous batched call's plans (checked on the device)."""
    _check(lib().bires_set_plan_cache(1 if enable else 0), "bires_set_plan_cache")


def plan_cache_stats():
    """(calls that reused plans, reuses undone by a statistics mismatch)."""
    h = ctypes.c_int64()
    m = ctypes.c_int64()
    _check(lib().bires_plan_cache_stats(ctypes.byref(h), ctypes.byref(m)), "bires_plan_cache_stats")
    return h.value, m.value


def set_graphs(enable):
    """Replay each batched call's device sequence as a captured HIP graph."""
    _check(lib().bires_set_graphs(1 if enable else 0), "bires_set_graphs")


def graph_stats():
    """(graphs captured, cached graphs replayed) since the library was set up."""
    c = ctypes.c_int64()
    r = ctypes.c_int64()
    _check(lib().bires_graph_stats(ctypes.byref(c), ctypes.byref(r)), "bires_graph_stats")
    return c.value, r.value


def set_timing(enable):
    _check(lib().bires_set_timing(1 if enable else 0), "bires_set_timing")


def kernel_time():
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().bires_kernel_time(ctypes.byref(ms), ctypes.byref(n)), "bires_kernel_time")
    return ms.value, n.value


HOST_PHASES = ("setup", "scan_submit", "scan_wait", "plan", "upload_and_launch", "device_wait_and_results")


def host_time():
    """Host microseconds per phase of the batched calls timed since the last
    set_timing (dict keyed by HOST_PHASES) and the number of calls."""
    us = (ctypes.c_double * len(HOST_PHASES))()
    n = ctypes.c_int64()
    _check(lib().bires_host_time(us, ctypes.byref(n)), "bires_host_time")
    return dict(zip(HOST_PHASES, list(us))), n.value


# ----------------------------------------------------------------------------
# device-memory entry points (inputs and outputs are torch tensors in HBM)

def _torch_stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class DeviceBatch:
    """A prepared batch of jobs whose inputs and outputs live in device memory.

    jobs: list of (kind, F, G, var) like resultant_batch.  The descriptors,
    input tensors and output tensors are built once; run() issues one
    bires_resultant_batch call (BIRES_MEM_DEVICE) on the given torch stream."""

    def __init__(self, jobs, device="cuda"):
        import torch
        n = len(jobs)
        self.n = n
        self.inputs = []
        self.fds = (Bipoly * n)()
        self.gds = (Bipoly * n)()
        self.kinds = (ctypes.c_int32 * n)()
        self.vars = (ctypes.c_int32 * n)()
        self.outs = (Upoly * n)()
        self.status = (ctypes.c_int32 * n)()
        self.out_tensors = []
        self.caps = []
        for i, (kind, F, G, var) in enumerate(jobs):
            k = _kind(kind)
            fdev = DeviceBipoly(F, device=device)
            gdev = DeviceBipoly(G, device=device) if k == KIND_RESULTANT else fdev
            self.inputs.append((fdev, gdev))
            self.fds[i] = fdev.desc()
            self.gds[i] = gdev.desc()
            self.kinds[i] = k
            self.vars[i] = _var(var)
            deg, L = _bounds(k, self.fds[i], self.gds[i], self.vars[i])
            t = torch.zeros((deg + 1, L), dtype=torch.int32, device=device)
            self.out_tensors.append(t)
            self.caps.append((deg, L))

    def _reset_outs(self):
        if not hasattr(self, "_outs_template"):
            self._outs_template = (Upoly * self.n)()
            for i, (deg, L) in enumerate(self.caps):
                self._outs_template[i] = Upoly(deg, L, self.out_tensors[i].data_ptr())
        ctypes.memmove(self.outs, self._outs_template, ctypes.sizeof(self.outs))

    def run(self, stream=None):
        self._reset_outs()
        code = lib().bires_resultant_batch(self.n, self.fds, self.gds, self.kinds, self.vars, self.outs,
                                           self.status, MEM_DEVICE, _torch_stream(stream))
        _check(code, "bires_resultant_batch")
        return code

    def run_async(self, stream=None):
        """Plans the batch and queues its device work (bires_resultant_batch_async),
        returning without waiting for the device; wait() collects it.  With
        stream (a torch stream) the work is queued there, after what is queued
        before; without one it goes to the library stream and the inputs must
        be complete.
        One call per DeviceBatch may be in flight: its descriptors and output
        tensors belong to that call until wait()."""
        if getattr(self, "_ticket", None) is not None:
            raise RuntimeError("a call of this batch is still in flight")
        self._reset_outs()
        t = ctypes.c_uint64()
        _check(lib().bires_resultant_batch_async(self.n, self.fds, self.gds, self.kinds, self.vars, self.outs,
                                                 self.status, MEM_DEVICE,
                                                 None if stream is None else _torch_stream(stream), ctypes.byref(t)),
               "bires_resultant_batch_async")
        self._ticket = t.value
        return t.value

    def wait(self):
        """Blocks until the call queued by run_async has finished."""
        t, self._ticket = getattr(self, "_ticket", None), None
        if t is None:
            raise RuntimeError("no call of this batch in flight")
        code = lib().bires_batch_wait(t)
        _check(code, "bires_batch_wait")
        return code

    def autotune(self, reps=3, stream=None):
        """Times this batch under each schedule; AUTO then uses the fastest. Returns its name."""
        self._reset_outs()
        chosen = ctypes.c_int32()
        _check(lib().bires_autotune(self.n, self.fds, self.gds, self.kinds, self.vars, self.outs, self.status,
                                    MEM_DEVICE, _torch_stream(stream), reps, ctypes.byref(chosen)),
               "bires_autotune")
        return {0: "staged", 1: "fused", 3: "schur"}[chosen.value]

    def run_each(self, stream=None):
        """The plain path: one single-job call per job (bires_resultant / bires_discriminant /
        bires_polar_resultant)."""
        s = _torch_stream(stream)
        self._reset_outs()
        for i in range(self.n):
            if self.kinds[i] == KIND_RESULTANT:
                code = lib().bires_resultant(ctypes.byref(self.fds[i]), ctypes.byref(self.gds[i]), self.vars[i],
                                             ctypes.byref(self.outs[i]), MEM_DEVICE, s)
            elif self.kinds[i] == KIND_DISCRIMINANT:
                code = lib().bires_discriminant(ctypes.byref(self.fds[i]), self.vars[i], ctypes.byref(self.outs[i]),
                                                MEM_DEVICE, s)
            else:
                code = lib().bires_polar_resultant(ctypes.byref(self.fds[i]), self.vars[i],
                                                   ctypes.byref(self.outs[i]), MEM_DEVICE, s)
            _check(code, "single-job call")

    def results(self):
        """Results as lists of Python ints (copies the output tensors to the host)."""
        res = []
        for i in range(self.n):
            deg = self.outs[i].degree
            arr = self.out_tensors[i][: deg + 1].cpu().numpy().view(np.uint32)
            res.append(limbs_to_ints(arr) if deg >= 0 else [])
        return res


def device_info():
    """(compute units, peak clock kHz, LDS bytes per block, HBM bytes) of the current device."""
    cu = ctypes.c_int32()
    clk = ctypes.c_int32()
    lds = ctypes.c_int64()
    hbm = ctypes.c_int64()
    _check(lib().bires_device_info(ctypes.byref(cu), ctypes.byref(clk), ctypes.byref(lds), ctypes.byref(hbm)),
           "bires_device_info")
    return {"cus": cu.value, "clock_khz": clk.value, "lds_per_block": lds.value, "hbm_bytes": hbm.value}


class Server:
    """Continuous-batching server (bires_server_*): submit() returns a ticket
    at once; wait() returns (result, latency in seconds)."""

    def __init__(self, hbm_budget_bytes=8 << 30, max_slots=512):
        h = ctypes.c_void_p()
        _check(lib().bires_server_create(hbm_budget_bytes, max_slots, ctypes.byref(h)), "bires_server_create")
        self.h = h

    def submit(self, kind, F, G=None, var="y"):
        k = _kind(kind)
        fa = bipoly_array(F)
        ga = bipoly_array(G) if k == KIND_RESULTANT else fa
        t = ctypes.c_uint64()
        _check(lib().bires_server_submit(self.h, k, _var(var), ctypes.byref(_desc(fa)), ctypes.byref(_desc(ga)),
                                         ctypes.byref(t)), "bires_server_submit")
        self._caps = getattr(self, "_caps", {})
        self._caps[t.value] = _bounds(k, _desc(fa), _desc(ga), _var(var))
        return t.value

    def wait(self, ticket, timeout=-1.0):
        deg, L = self._caps.pop(ticket)
        out = np.zeros((deg + 1, L), dtype=np.uint32)
        od = Upoly(deg, L, out.ctypes.data)
        lat = ctypes.c_double()
        _check(lib().bires_server_wait(self.h, ticket, ctypes.byref(od), timeout, ctypes.byref(lat)),
               "bires_server_wait")
        return limbs_to_ints(out[: od.degree + 1]), lat.value

    def close(self):
        if self.h:
            _check(lib().bires_server_destroy(self.h), "bires_server_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
