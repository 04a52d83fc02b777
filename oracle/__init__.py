"""FP64 CPU oracle for the batched band-SLAE methods (TEST INFRASTRUCTURE).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The product library never does, and this package never
imports the product.  Every routine is a thin ctypes call into
band_oracle.cpp, a plain serial C++ transcription of the methods of
Veneva & Ayriyan (arXiv:1804.09666): NPDM / NTDM / MNPDM (Sec. 1), ILU(0) and
the Stone method SIP (Sec. 2, Algorithm 1), and the Hotelling-Bodewig inverse
iteration (Appendix).

Arrays are float64 numpy arrays in *system-contiguous* layout: one system is a
1-D array of length n, a batch is a 2-D array [batch, n].  Conversion from the
batch-interleaved device layout ([n, ld], system s in column s) is the
caller's business (`np.ascontiguousarray(a[:, :batch].T)`).
"""
import ctypes
import os

import numpy as np

from . import build_oracle

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64 = ctypes.c_int64
_int = ctypes.c_int

_LIBS = {}


def _load(count: bool = False):
    key = "count" if count else "plain"
    if key in _LIBS:
        return _LIBS[key]
    path = build_oracle.LIB_COUNT if count else build_oracle.LIB
    if not os.path.exists(path):
        build_oracle.build(force=False)
    _LIBS[key] = bind(ctypes.CDLL(path))
    return _LIBS[key]


def bind(lib):
    """Declare the C signatures on a loaded oracle library (also used by the
    tests that load deliberately broken copies of it)."""
    sig = {
        "orc_npdm": (_int, [_i64] + [_dp] * 8),
        "orc_ntdm": (_int, [_i64] + [_dp] * 6),
        "orc_mnpdm": (_int, [_i64, _dp, _dp, _dp, _i64, _i64p, _dp, _dp, _dp, _dp]),
        "orc_ilu0_band": (_int, [_i64] + [_dp] * 9),
        "orc_ilu0_pattern_dense": (_int, [_i64, _dp, _u8p]),
        "orc_band_lu_solve": (_int, [_i64] + [_dp] * 7),
        "orc_hb_matrix": (_int, [_i64, _dp, _int, _dp]),
        "orc_hb_lower_apply": (_int, [_i64, _dp, _dp, _int, _dp, _dp]),
        "orc_hb_upper_apply": (_int, [_i64, _dp, _dp, _dp, _int, _dp, _dp]),
        "orc_sip": (_int, [_i64] + [_dp] * 10 + [ctypes.c_double, _int, _int, _int,
                                                 _dp, ctypes.POINTER(_int), _dp]),
        "orc_dense_solve": (_int, [_i64, _dp, _dp, _dp, _int]),
        "orc_npdm_batch": (None, [_i64, _i64] + [_dp] * 7 + [_i32p, _int]),
        "orc_ntdm_batch": (None, [_i64, _i64] + [_dp] * 5 + [_i32p, _int]),
        "orc_ilu0_band_batch": (None, [_i64, _i64] + [_dp] * 9 + [_i32p, _int]),
        "orc_sip_batch": (None, [_i64, _i64] + [_dp] * 6 +
                          [ctypes.c_double, _int, _int, _int, _dp, _i32p, _dp, _i32p, _int]),
        "orc_flops_get": (ctypes.c_longlong, []),
        "orc_flops_reset": (None, []),
        "orc_max_threads": (_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def max_threads() -> int:
    return _load().orc_max_threads()


# ----------------------------------------------------------------- direct ---
def npdm(e, c, d, a, b, y, *, return_mu=False, lib=None):
    """NPDM (Sec. 1) on one system (1-D) or a batch (2-D [batch, n]).

    Returns (x, info) or (x, info, mu).  info is 0 or the 1-based row of the
    first zero / non-finite pivot."""
    lib = lib or _load()
    arrs = [_f64(v) for v in (e, c, d, a, b, y)]
    two_d = arrs[5].ndim == 2
    if not two_d:
        arrs = [v[None, :] for v in arrs]
    bsz, n = arrs[5].shape
    x = np.zeros((bsz, n))
    mu = np.zeros((bsz, n))
    info = np.zeros(bsz, dtype=np.int32)
    for s in range(bsz):
        info[s] = lib.orc_npdm(n, *[_p(v[s]) for v in arrs], _p(x[s]), _p(mu[s]))
    if not two_d:
        x, mu, info = x[0], mu[0], int(info[0])
    return (x, info, mu) if return_mu else (x, info)


def ntdm(c, d, a, y, *, return_mu=False, lib=None):
    """NTDM (Thomas, Sec. 1) on one system or a batch."""
    lib = lib or _load()
    arrs = [_f64(v) for v in (c, d, a, y)]
    two_d = arrs[3].ndim == 2
    if not two_d:
        arrs = [v[None, :] for v in arrs]
    bsz, n = arrs[3].shape
    x = np.zeros((bsz, n))
    mu = np.zeros((bsz, n))
    info = np.zeros(bsz, dtype=np.int32)
    for s in range(bsz):
        info[s] = lib.orc_ntdm(n, *[_p(v[s]) for v in arrs], _p(x[s]), _p(mu[s]))
    if not two_d:
        x, mu, info = x[0], mu[0], int(info[0])
    return (x, info, mu) if return_mu else (x, info)


def mnpdm(c, d, a, rows, e_at, b_at, y, *, lib=None):
    """MNPDM (Sec. 1) on ONE system; outer diagonals as a row-ascending list."""
    lib = lib or _load()
    c, d, a, y = (_f64(v) for v in (c, d, a, y))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    e_at, b_at = _f64(e_at), _f64(b_at)
    n = y.shape[0]
    x = np.zeros(n)
    info = lib.orc_mnpdm(n, _p(c), _p(d), _p(a), rows.shape[0],
                         rows.ctypes.data_as(_i64p), _p(e_at), _p(b_at), _p(y), _p(x))
    return x, int(info)


def ilu0_band(e, c, d, a, b, *, lib=None):
    """ILU(0) = band Doolittle (Sec. 2) of one system: (l2, l1, u0, u1, info)."""
    lib = lib or _load()
    arrs = [_f64(v) for v in (e, c, d, a, b)]
    n = arrs[2].shape[0]
    out = [np.zeros(n) for _ in range(4)]
    info = lib.orc_ilu0_band(n, *[_p(v) for v in arrs], *[_p(v) for v in out])
    return (*out, int(info))


def ilu0_pattern_dense(A, pattern, *, lib=None):
    """Textbook ILU(0) (IKJ elimination restricted to the pattern) on a dense
    matrix.  Returns (L, U, info): L unit lower, U upper."""
    lib = lib or _load()
    M = np.array(A, dtype=np.float64, order="C", copy=True)
    pat = np.ascontiguousarray(pattern, dtype=np.uint8)
    n = M.shape[0]
    info = lib.orc_ilu0_pattern_dense(n, _p(M), pat.ctypes.data_as(_u8p))
    L = np.tril(M, -1) + np.eye(n)
    U = np.triu(M)
    return L, U, int(info)


def band_lu_solve(l2, l1, u0, u1, b, y, *, lib=None):
    lib = lib or _load()
    arrs = [_f64(v) for v in (l2, l1, u0, u1, b, y)]
    n = arrs[5].shape[0]
    x = np.zeros(n)
    info = lib.orc_band_lu_solve(n, *[_p(v) for v in arrs], _p(x))
    return x, int(info)


# ------------------------------------------------------ Hotelling-Bodewig ---
def hb_matrix(T, s, *, lib=None):
    """s steps of X_{j+1} = X_j (2I - T X_j), X_0 = diag(T)^-1 (Appendix)."""
    lib = lib or _load()
    T = np.array(T, dtype=np.float64, order="C")
    n = T.shape[0]
    X = np.zeros((n, n))
    info = lib.orc_hb_matrix(n, _p(T), int(s), _p(X))
    if info != 0:
        raise ValueError(f"zero diagonal at row {info - 1}")
    return X


def hb_lower_apply(l2, l1, s, v, *, lib=None):
    lib = lib or _load()
    l2, l1, v = _f64(l2), _f64(l1), _f64(v)
    out = np.zeros_like(v)
    if lib.orc_hb_lower_apply(v.shape[0], _p(l2), _p(l1), int(s), _p(v), _p(out)) != 0:
        raise ValueError("bad s")
    return out


def hb_upper_apply(u0, u1, b, s, v, *, lib=None):
    lib = lib or _load()
    u0, u1, b, v = _f64(u0), _f64(u1), _f64(b), _f64(v)
    out = np.zeros_like(v)
    if lib.orc_hb_upper_apply(v.shape[0], _p(u0), _p(u1), _p(b), int(s), _p(v), _p(out)) != 0:
        raise ValueError("bad s")
    return out


# ---------------------------------------------------------------- SIP -------
def sip(e, c, d, a, b, y, *, tol, max_iter, s_L=-1, s_U=-1, x0=None,
        factors=None, lib=None):
    """Stone method (Sec. 2, Algorithm 1) on ONE system.

    Returns (x, iters, relres, status); status 0 converged, -1 max_iter,
    -2 diverged, i+1 bad ILU(0) pivot, -3 bad argument."""
    lib = lib or _load()
    arrs = [_f64(v) for v in (e, c, d, a, b, y)]
    n = arrs[5].shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    f = [None] * 4 if factors is None else [_f64(v) for v in factors]
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    st = lib.orc_sip(n, *[_p(v) for v in arrs], *[_p(v) for v in f], float(tol),
                     int(max_iter), int(s_L), int(s_U), _p(x), ctypes.byref(it),
                     ctypes.byref(rr))
    return x, it.value, rr.value, int(st)


def dense_solve(A, y, pivot=True, *, lib=None):
    lib = lib or _load()
    M = np.array(A, dtype=np.float64, order="C", copy=True)
    r = np.array(y, dtype=np.float64, copy=True)
    x = np.zeros_like(r)
    info = lib.orc_dense_solve(M.shape[0], _p(M), _p(r), _p(x), int(bool(pivot)))
    return x, int(info)


# -------------------------------------------------------- batch drivers -----
def npdm_batch(e, c, d, a, b, y, nthreads=0, *, lib=None):
    """NPDM over a [batch, n] batch with OpenMP over systems."""
    lib = lib or _load()
    arrs = [_f64(v) for v in (e, c, d, a, b, y)]
    bsz, n = arrs[5].shape
    x = np.zeros((bsz, n))
    info = np.zeros(bsz, dtype=np.int32)
    lib.orc_npdm_batch(n, bsz, *[_p(v) for v in arrs], _p(x),
                       info.ctypes.data_as(_i32p), int(nthreads))
    return x, info


def ntdm_batch(c, d, a, y, nthreads=0, *, lib=None):
    lib = lib or _load()
    arrs = [_f64(v) for v in (c, d, a, y)]
    bsz, n = arrs[3].shape
    x = np.zeros((bsz, n))
    info = np.zeros(bsz, dtype=np.int32)
    lib.orc_ntdm_batch(n, bsz, *[_p(v) for v in arrs], _p(x),
                       info.ctypes.data_as(_i32p), int(nthreads))
    return x, info


def ilu0_band_batch(e, c, d, a, b, nthreads=0, *, lib=None):
    lib = lib or _load()
    arrs = [_f64(v) for v in (e, c, d, a, b)]
    bsz, n = arrs[2].shape
    out = [np.zeros((bsz, n)) for _ in range(4)]
    info = np.zeros(bsz, dtype=np.int32)
    lib.orc_ilu0_band_batch(n, bsz, *[_p(v) for v in arrs], *[_p(v) for v in out],
                            info.ctypes.data_as(_i32p), int(nthreads))
    return (*out, info)


def sip_batch(e, c, d, a, b, y, *, tol, max_iter, s_L=-1, s_U=-1, x0=None,
              nthreads=0, lib=None):
    lib = lib or _load()
    arrs = [_f64(v) for v in (e, c, d, a, b, y)]
    bsz, n = arrs[5].shape
    x = np.zeros((bsz, n)) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    iters = np.zeros(bsz, dtype=np.int32)
    relres = np.zeros(bsz)
    status = np.zeros(bsz, dtype=np.int32)
    lib.orc_sip_batch(n, bsz, *[_p(v) for v in arrs], float(tol), int(max_iter),
                      int(s_L), int(s_U), _p(x), iters.ctypes.data_as(_i32p),
                      _p(relres), status.ctypes.data_as(_i32p), int(nthreads))
    return x, iters, relres, status


# ------------------------------------------------------------ op counts -----
def count_flops(name, *args, **kwargs):
    """Run oracle routine `name` on the counting build; return its flop count."""
    lib = _load(count=True)
    lib.orc_flops_reset()
    globals()[name](*args, lib=lib, **kwargs)
    return int(lib.orc_flops_get())
