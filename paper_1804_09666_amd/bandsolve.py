"""Python binding of libbandsolve (include/bandsolve.h).

Argument marshalling only: tensors are checked for device, dtype, layout and
shape, their device pointers and the current HIP stream are handed to the C
ABI, and any non-zero status becomes a BandSolveError.  Every step of every
solve runs in the library's HIP kernels; this module computes nothing.  If the
library is not built, loading fails loudly -- there is no fallback.

Layout: every per-row array is a 2-D float64 (or float32) tensor [n, ld] in
the batch-interleaved layout -- element (row i, system s) at [i, s] -- with
systems 0..batch-1 in the first `batch` columns (batch <= ld).  Diagonals are
passed as a 5-list (e, c, d, a, b); for tridiagonal systems (kind 3) e and b
may be None.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbandsolve.so")

BS_OK, BS_EINVAL, BS_ELAUNCH, BS_EWORKSPACE, BS_ENODEV = range(5)
BS_F64, BS_F32 = 0, 1
NOALLOC_SCRATCH_BYTES = 128 << 20     # BS_NOALLOC_SCRATCH_BYTES of include/bandsolve.h
OP_FACTOR, OP_SOLVE, OP_SOLVE_FACTORED, OP_MNPDM, OP_SIP, OP_REFINE, OP_ADI = range(7)

EXPORTED = ("bs_status_str", "bs_version", "bs_workspace_bytes", "bs_set_option",
            "bs_get_option", "bs_part_variant", "band_factor", "band_solve",
            "band_solve_refine", "band_solve_adi", "band_solve_mnpdm", "sip_solve",
            "bs_varlen_variants",
            "bs_varlen_variant_shape", "bs_varlen_layout", "bs_varlen_workspace_bytes",
            "band_solve_varlen", "bs_varlen_tune", "bs_pack_interleave", "bs_unpack_interleave",
            "bs_stream_probe", "band_solve_noalloc",
            "hb_inverse_band_workspace_bytes", "hb_inverse_band")
(OPT_DIRECT_PATH, OPT_PART_PD_VARIANT, OPT_PART_TD_VARIANT, OPT_SIP_PATH, OPT_EXCHANGE_WAIT_US,
 OPT_F32_STATE) = range(6)
PATH_AUTO, PATH_LANE, PATH_PART = range(3)


class VarlenInfo(ctypes.Structure):
    """bs_varlen_info of include/bandsolve.h."""
    _fields_ = [("count", ctypes.c_int64), ("groups", ctypes.c_int64), ("elems", ctypes.c_int64),
                ("tiles", ctypes.c_int64 * 4), ("table_bytes", ctypes.c_size_t),
                ("nmax", ctypes.c_int64)]


class BandSolveError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {status_str(status)}")


_lib = None


def load():
    """Load libbandsolve.so (built by __graft_entry__.build()).  No fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    vp5 = ctypes.c_void_p * 5
    vp3 = ctypes.c_void_p * 3
    sig = {
        "bs_status_str": (ctypes.c_char_p, [i32]),
        "bs_version": (i32, []),
        "bs_workspace_bytes": (sz, [i32, i32, i32, i64, i64, i64]),
        "bs_set_option": (i32, [i32, i64]),
        "bs_get_option": (i64, [i32]),
        "bs_part_variant": (i32, [i32, i32, ctypes.POINTER(i32)]),
        "band_factor": (i32, [i32, i32, i64, i64, i64, vp5, vp, vp, vp]),
        "band_solve": (i32, [i32, i32, i64, i64, i64, vp5, vp, vp, vp, vp, vp, sz, vp]),
        "band_solve_refine": (i32, [i32, i64, i64, i64, vp5, vp, vp, ctypes.c_double, i32,
                                    vp, vp, vp, vp, sz, vp]),
        "band_solve_adi": (i32, [i32, i64, i64, i64, ctypes.c_double, vp, vp, vp, vp, sz, vp]),
        "band_solve_mnpdm": (i32, [i32, i64, i64, i64, vp3, i32, vp, vp, vp, vp, vp,
                                   vp, vp, sz, vp]),
        "sip_solve": (i32, [i32, i64, i64, i64, vp5, vp, vp, vp, ctypes.c_double, i32,
                            i32, i32, vp, vp, vp, vp, sz, vp]),
    }
    vip = ctypes.POINTER(VarlenInfo)
    sig.update({
        "bs_varlen_variants": (i32, []),
        "bs_varlen_variant_shape": (i32, [i32, ctypes.POINTER(i32)]),
        "bs_varlen_layout": (i32, [i64, vp, vp, vp, vp, vip]),
        "bs_varlen_workspace_bytes": (sz, [i32, vip, i32]),
        "band_solve_varlen": (i32, [i32, vip, vp, i32, vp5, vp, vp, vp, vp, sz, vp]),
        "bs_varlen_tune": (i32, [i32, vip, vp, vp5, vp, vp, vp, vp, sz, i32, vp, vp, vp]),
        "bs_stream_probe": (i32, [i64, i32, ctypes.c_void_p * 6, vp, vp]),
        "bs_pack_interleave": (i32, [i64, i64, vp, i64, vp, i64, vp]),
        "band_solve_noalloc": (i32, [i32, i32, i64, i64, i64, vp5, vp, vp, vp, vp]),
        "bs_unpack_interleave": (i32, [i64, i64, vp, i64, vp, i64, vp]),
        "hb_inverse_band_workspace_bytes": (sz, [i32, i64, i64, i64, i32, i32]),
        "hb_inverse_band": (i32, [i32, i64, i64, i64, vp5, vp, i32, i32, vp, vp, vp, sz, vp]),
    })
    for name, (res, args) in sig.items():
        if not hasattr(lib, name):
            raise RuntimeError(f"{LIB_PATH} does not export {name}; rebuild it")
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    lib.VP5 = vp5
    lib.VP3 = vp3
    _lib = lib
    return lib


def status_str(status):
    return load().bs_status_str(int(status)).decode()


def set_option(key, value):
    st = load().bs_set_option(int(key), int(value))
    if st != BS_OK:
        raise BandSolveError(st, f"bs_set_option({key}, {value})")


def get_option(key):
    return int(load().bs_get_option(int(key)))


def part_variants(kind):
    """[(M, PW, G, TMAX), ...] of the compiled split-row variants of `kind`."""
    out = []
    shape = (ctypes.c_int32 * 4)()
    while load().bs_part_variant(kind, len(out), shape) == BS_OK:
        out.append(tuple(shape))
    return out


def pack_interleave(lines, ld=None, out=None, stream=None):
    """[batch, n] system-contiguous FP64 lines (row stride >= n) -> the
    interleaved [n, ld] layout of the solvers."""
    batch, n = lines.shape
    if lines.dtype != torch.float64 or lines.stride(1) != 1:
        raise ValueError("pack_interleave: float64 lines with unit column stride")
    ld = batch if ld is None else ld
    out = torch.empty((n, ld), dtype=torch.float64, device=lines.device) if out is None else out
    if out.shape != (n, ld) or not out.is_contiguous():
        raise ValueError("pack_interleave: out must be a contiguous [n, ld] tensor")
    _raise(load().bs_pack_interleave(n, batch, _ptr(lines), lines.stride(0), _ptr(out), ld,
                                     _stream(stream)), "bs_pack_interleave")
    return out


def unpack_interleave(x, batch, out=None, stream=None):
    """The interleaved [n, ld] layout -> [batch, n] system-contiguous lines."""
    n, ld = x.shape
    if x.dtype != torch.float64 or not x.is_contiguous():
        raise ValueError("unpack_interleave: a contiguous float64 [n, ld] tensor")
    out = torch.empty((batch, n), dtype=torch.float64, device=x.device) if out is None else out
    if out.shape[0] != batch or out.shape[1] != n or out.stride(1) != 1:
        raise ValueError("unpack_interleave: out must be [batch, n] with unit column stride")
    _raise(load().bs_unpack_interleave(n, batch, _ptr(x), ld, _ptr(out), out.stride(0),
                                       _stream(stream)), "bs_unpack_interleave")
    return out


def stream_probe(inputs, out, stream=None):
    """out = sum(inputs) elementwise in one streaming pass (a measurement of the
    HBM ceiling of the solvers' traffic pattern; 1..6 FP64 inputs)."""
    lib = load()
    arr = (ctypes.c_void_p * 6)(*[_ptr(t) for t in inputs])
    st = lib.bs_stream_probe(out.numel(), len(inputs), arr, _ptr(out), _stream(stream))
    _raise(st, "bs_stream_probe")
    return out


def workspace_bytes(op, kind, n, batch, dtype=BS_F64, ld=None):
    ld = batch if ld is None else ld
    v = load().bs_workspace_bytes(op, kind, dtype, n, batch, ld)
    if v == ctypes.c_size_t(-1).value:
        raise BandSolveError(BS_EINVAL, "bs_workspace_bytes")
    return v


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check2d(t, name, n, dtype):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype or t.dim() != 2 or t.shape[0] != n or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape [n={n}, ld]")
    return t.shape[1]


def _dtype_code(dtype):
    return {torch.float64: BS_F64, torch.float32: BS_F32}[dtype]


def _prep(diags, rhs, kind, batch):
    d = diags[2]
    n = d.shape[0]
    dtype = d.dtype
    if kind is None:
        kind = 5 if (diags[0] is not None and diags[4] is not None) else 3
    need = range(5) if kind == 5 else (1, 2, 3)
    ld = None
    for k in need:
        l_k = _check2d(diags[k], "diags[%d]" % k, n, dtype)
        if ld is None:
            ld = l_k
        elif l_k != ld:
            raise ValueError("all arrays must share one leading dimension")
    if rhs is not None and _check2d(rhs, "rhs", n, dtype) != ld:
        raise ValueError("rhs leading dimension differs")
    batch = ld if batch is None else int(batch)
    return kind, n, ld, batch, dtype


def _ws(nbytes, device):
    """Workspace for one call; zero-filled (the split-row solver's counters
    must start at zero)."""
    if nbytes == 0:
        return None
    return torch.zeros((nbytes + 7) // 8, dtype=torch.float64, device=device)


def _raise(st, what):
    if st != BS_OK:
        raise BandSolveError(st, what)


def factor(diags, *, kind=None, batch=None, out=None, info=None, stream=None):
    """ILU(0) (band Doolittle) of every system -> (factors [nf, n, ld], info)."""
    lib = load()
    kind, n, ld, batch, dtype = _prep(diags, None, kind, batch)
    nf = 4 if kind == 5 else 2
    dev = diags[2].device
    out = torch.empty((nf, n, ld), dtype=dtype, device=dev) if out is None else out
    info = torch.empty(batch, dtype=torch.int32, device=dev) if info is None else info
    st = lib.band_factor(kind, _dtype_code(dtype), n, batch, ld,
                         lib.VP5(*[_ptr(t) for t in diags]), _ptr(out), _ptr(info),
                         _stream(stream))
    _raise(st, "band_factor")
    return out, info


def solve(diags, rhs, x=None, *, kind=None, batch=None, factors=None, info=None,
          workspace=None, stream=None):
    """x = A^{-1} rhs for every system (NPDM / NTDM, or substitution with
    `factors` from factor()).  Returns (x, info)."""
    lib = load()
    kind, n, ld, batch, dtype = _prep(diags, rhs, kind, batch)
    dev = rhs.device
    x = torch.empty_like(rhs) if x is None else x
    _check2d(x, "x", n, dtype)
    info = torch.empty(batch, dtype=torch.int32, device=dev) if info is None else info
    op = OP_SOLVE if factors is None else OP_SOLVE_FACTORED
    nbytes = workspace_bytes(op, kind, n, batch, _dtype_code(dtype), ld)
    if workspace is None:
        workspace = _ws(nbytes, dev)
    st = lib.band_solve(kind, _dtype_code(dtype), n, batch, ld,
                        lib.VP5(*[_ptr(t) for t in diags]), _ptr(factors), _ptr(rhs),
                        _ptr(x), _ptr(info), _ptr(workspace),
                        0 if workspace is None else workspace.numel() * workspace.element_size(),
                        _stream(stream))
    _raise(st, "band_solve")
    return x, info


def solve_noalloc(diags, rhs, x=None, *, kind=None, batch=None, info=None, stream=None):
    """band_solve_noalloc: the fused solve with the library's static scratch
    (no workspace).  Returns (x, info)."""
    lib = load()
    kind, n, ld, batch, dtype = _prep(diags, rhs, kind, batch)
    x = torch.empty_like(rhs) if x is None else x
    _check2d(x, "x", n, dtype)
    info = torch.empty(batch, dtype=torch.int32, device=rhs.device) if info is None else info
    st = lib.band_solve_noalloc(kind, _dtype_code(dtype), n, batch, ld,
                                lib.VP5(*[_ptr(t) for t in diags]), _ptr(rhs), _ptr(x),
                                _ptr(info), _stream(stream))
    _raise(st, "band_solve_noalloc")
    return x, info


def refine(diags, rhs, x=None, *, tol=1e-12, max_steps=8, kind=None, batch=None,
           workspace=None, stream=None):
    """FP32-storage NPDM / NTDM with FP64 iterative refinement on FP64 data
    -> (x, steps, relres, info).  x must not alias rhs."""
    lib = load()
    kind, n, ld, batch, dtype = _prep(diags, rhs, kind, batch)
    if dtype != torch.float64:
        raise ValueError("refine takes float64 diagonals and right-hand side")
    dev = rhs.device
    x = torch.empty_like(rhs) if x is None else x
    _check2d(x, "x", n, dtype)
    steps = torch.empty(batch, dtype=torch.int32, device=dev)
    relres = torch.empty(batch, dtype=torch.float64, device=dev)
    info = torch.empty(batch, dtype=torch.int32, device=dev)
    nbytes = workspace_bytes(OP_REFINE, kind, n, batch, BS_F64, ld)
    workspace = _ws(nbytes, dev) if workspace is None else workspace
    st = lib.band_solve_refine(kind, n, batch, ld, lib.VP5(*[_ptr(t) for t in diags]),
                               _ptr(rhs), _ptr(x), float(tol), int(max_steps), _ptr(steps),
                               _ptr(relres), _ptr(info), _ptr(workspace),
                               workspace.numel() * workspace.element_size(), _stream(stream))
    _raise(st, "band_solve_refine")
    return x, steps, relres, info


def solve_adi(v, r, x=None, *, kind=5, batch=None, info=None, workspace=None, stream=None):
    """One ADI sweep assembled in the kernel: lines are the columns of the
    [n, ld] float64 field v (see band_solve_adi).  Returns (x, info)."""
    lib = load()
    n = v.shape[0]
    ld = _check2d(v, "v", n, torch.float64)
    batch = ld if batch is None else int(batch)
    x = torch.empty_like(v) if x is None else x
    _check2d(x, "x", n, torch.float64)
    info = torch.empty(batch, dtype=torch.int32, device=v.device) if info is None else info
    nbytes = workspace_bytes(OP_ADI, kind, n, batch, BS_F64, ld)
    workspace = _ws(nbytes, v.device) if workspace is None else workspace
    st = lib.band_solve_adi(kind, n, batch, ld, float(r), _ptr(v), _ptr(x), _ptr(info),
                            _ptr(workspace),
                            0 if workspace is None else workspace.numel() * workspace.element_size(),
                            _stream(stream))
    _raise(st, "band_solve_adi")
    return x, info


def solve_mnpdm(cda, outer_row, outer_e, outer_b, rhs, x=None, *, batch=None,
                info=None, workspace=None, stream=None):
    """MNPDM: c, d, a as [n, ld] tensors; the outer entries as [kmax, ld]
    tensors (int32 rows, -1 = unused; float64 e and b values)."""
    lib = load()
    c, d, a = cda
    n = d.shape[0]
    ld = _check2d(d, "d", n, torch.float64)
    for t, nm in ((c, "c"), (a, "a"), (rhs, "rhs")):
        if _check2d(t, nm, n, torch.float64) != ld:
            raise ValueError("leading dimension mismatch")
    batch = ld if batch is None else int(batch)
    kmax = 0 if outer_row is None else outer_row.shape[0]
    if kmax:
        for t, dt in ((outer_row, torch.int32), (outer_e, torch.float64), (outer_b, torch.float64)):
            if t.dtype != dt or t.shape != (kmax, ld) or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("outer lists must be contiguous [kmax, ld] device tensors")
    dev = rhs.device
    x = torch.empty_like(rhs) if x is None else x
    info = torch.empty(batch, dtype=torch.int32, device=dev) if info is None else info
    nbytes = workspace_bytes(OP_MNPDM, 5, n, batch, ld=ld)
    workspace = _ws(nbytes, dev) if workspace is None else workspace
    st = lib.band_solve_mnpdm(BS_F64, n, batch, ld, lib.VP3(*[_ptr(t) for t in cda]), kmax,
                              _ptr(outer_row) if kmax else None,
                              _ptr(outer_e) if kmax else None,
                              _ptr(outer_b) if kmax else None, _ptr(rhs), _ptr(x),
                              _ptr(info), _ptr(workspace),
                              0 if workspace is None else workspace.numel() * workspace.element_size(),
                              _stream(stream))
    _raise(st, "band_solve_mnpdm")
    return x, info


def hb_band_width(kind, s, n):
    """Bandwidth of the HB iterate X_s of an ILU(0) factor: q (2^s - 1), q = 2
    (kind 5) or 1 (kind 3), at most n - 1."""
    return min(n - 1, (2 if kind == 5 else 1) * (2 ** s - 1))


def hb_inverse(diags, factors, *, s_L=None, s_U=None, kind=None, batch=None, workspace=None,
               out=None, stream=None):
    """Explicit banded HB iterates of the ILU(0) factors -> (XL, XU): XL[d, i, s]
    = X_L[i, i - d] (s_L steps), XU[d, i, s] = X_U[i, i + d] (s_U steps), each
    [K + 1, n, ld] (None where the step count is None).  out: optional
    (XL, XU) tensors of those shapes to write into."""
    lib = load()
    kind, n, ld, batch, dtype = _prep(diags, None, kind, batch)
    dev = diags[2].device
    sl = -1 if s_L is None else int(s_L)
    su = -1 if s_U is None else int(s_U)
    shapes = [None if v < 0 else (hb_band_width(kind, v, n) + 1, n, ld) for v in (sl, su)]
    if out is None:
        out = [None if sh is None else torch.zeros(sh, dtype=torch.float64, device=dev)
               for sh in shapes]
    XL, XU = out
    for t, sh, name in ((XL, shapes[0], "XL"), (XU, shapes[1], "XU")):
        if (t is None) != (sh is None) or (t is not None and (
                tuple(t.shape) != sh or t.dtype != torch.float64 or not t.is_contiguous())):
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape {sh}")
    nb = lib.hb_inverse_band_workspace_bytes(kind, n, batch, ld, max(sl, 0), max(su, 0))
    if nb == ctypes.c_size_t(-1).value:
        raise BandSolveError(BS_EINVAL, "hb_inverse_band_workspace_bytes")
    if workspace is None:
        workspace = _ws(nb, dev)
    st = lib.hb_inverse_band(kind, n, batch, ld, lib.VP5(*[_ptr(t) for t in diags]),
                             _ptr(factors), max(sl, 0), max(su, 0), _ptr(XL), _ptr(XU),
                             _ptr(workspace), workspace.numel() * workspace.element_size(),
                             _stream(stream))
    _raise(st, "hb_inverse_band")
    return XL, XU


def sip(diags, rhs, x0=None, *, tol, max_iter, s_L=-1, s_U=-1, factors=None,
        batch=None, x=None, workspace=None, stream=None):
    """Stone method over ILU(0) -> (x, iters, relres, info).  x0 (or x) is the
    start vector; zeros when both are None."""
    lib = load()
    kind, n, ld, batch, dtype = _prep(diags, rhs, 5, batch)
    dev = rhs.device
    if x is None:
        x = torch.zeros_like(rhs) if x0 is None else x0.clone()
    elif x0 is not None:
        x.copy_(x0)
    iters = torch.empty(batch, dtype=torch.int32, device=dev)
    relres = torch.empty(batch, dtype=torch.float64, device=dev)
    info = torch.empty(batch, dtype=torch.int32, device=dev)
    nbytes = workspace_bytes(OP_SIP, 5, n, batch, ld=ld)
    workspace = _ws(nbytes, dev) if workspace is None else workspace
    st = lib.sip_solve(BS_F64, n, batch, ld, lib.VP5(*[_ptr(t) for t in diags]),
                       _ptr(factors), _ptr(rhs), _ptr(x), float(tol), int(max_iter),
                       int(s_L), int(s_U), _ptr(iters), _ptr(relres), _ptr(info),
                       _ptr(workspace), workspace.numel() * workspace.element_size(),
                       _stream(stream))
    _raise(st, "sip_solve")
    return x, iters, relres, info


# ------------------------------------------------------------ uneven batches --
class Varlen:
    """Plan of an uneven batch (bs_varlen_layout): sizes -> group layout.
    offset[i]: element of row 0 of system i (row r at offset[i] + 16 r);
    slot[i]: its info entry.  The device table is uploaded once."""

    def __init__(self, n, device="cuda"):
        import numpy as np
        lib = load()
        n = np.ascontiguousarray(np.asarray(n, dtype=np.int64))
        self.count = n.size
        self.n = n
        self.info = VarlenInfo()
        self.offset = np.empty(n.size, dtype=np.int64)
        self.slot = np.empty(n.size, dtype=np.int32)
        st = lib.bs_varlen_layout(n.size, n.ctypes.data, self.offset.ctypes.data,
                                  self.slot.ctypes.data, None, ctypes.byref(self.info))
        if st != BS_OK:
            raise BandSolveError(st, "bs_varlen_layout")
        table = np.zeros(self.info.table_bytes, dtype=np.uint8)
        lib.bs_varlen_layout(n.size, n.ctypes.data, None, None, table.ctypes.data,
                             ctypes.byref(self.info))
        self.table = torch.from_numpy(table).to(device)
        self.elems = self.info.elems
        self.slots = self.info.groups * 16
        self.slot_sizes = np.zeros(self.slots, dtype=np.int64)   # length of the system in each slot
        self.slot_sizes[self.slot] = n

    def variants(self):
        lib = load()
        out, shape = [], (ctypes.c_int32 * 2)()
        for v in range(lib.bs_varlen_variants()):
            lib.bs_varlen_variant_shape(v, shape)
            out.append(tuple(shape))
        return out

    def workspace(self, kind, variant=None):
        lib = load()
        vs = range(lib.bs_varlen_variants()) if variant is None else [variant]
        nbytes = max(lib.bs_varlen_workspace_bytes(kind, ctypes.byref(self.info), v) for v in vs)
        return torch.empty(nbytes // 8 + 1, dtype=torch.float64, device=self.table.device)

    def pack(self, systems, fill=0.0):
        """Host list of 1-D arrays (system i's rows) -> flat float64 numpy array
        in the group layout."""
        import numpy as np
        out = np.full(self.elems, fill, dtype=np.float64)
        for i, v in enumerate(systems):
            out[self.offset[i] + 16 * np.arange(len(v))] = v
        return out

    def unpack(self, flat):
        """Inverse of pack for a host array."""
        import numpy as np
        return [flat[self.offset[i] + 16 * np.arange(self.n[i])] for i in range(self.count)]

    def solve(self, kind, diags, rhs, x=None, info=None, variant=0, workspace=None, stream=None):
        lib = load()
        x = torch.empty_like(rhs) if x is None else x
        info = torch.empty(self.slots, dtype=torch.int32, device=rhs.device) if info is None else info
        ws = self.workspace(kind, variant) if workspace is None else workspace
        st = lib.band_solve_varlen(kind, ctypes.byref(self.info), _ptr(self.table), variant,
                                   lib.VP5(*[_ptr(t) for t in diags]), _ptr(rhs), _ptr(x),
                                   _ptr(info), _ptr(ws), ws.numel() * ws.element_size(),
                                   _stream(stream))
        _raise(st, "band_solve_varlen")
        return x, info

    def tune(self, kind, diags, rhs, x, info, workspace, reps=5, stream=None):
        """Autotuner: (best variant, [ms per variant])."""
        lib = load()
        nv = lib.bs_varlen_variants()
        ms = (ctypes.c_float * nv)()
        best = ctypes.c_int32(-1)
        st = lib.bs_varlen_tune(kind, ctypes.byref(self.info), _ptr(self.table),
                                lib.VP5(*[_ptr(t) for t in diags]), _ptr(rhs), _ptr(x),
                                _ptr(info), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), int(reps), ms,
                                ctypes.byref(best), _stream(stream))
        _raise(st, "bs_varlen_tune")
        return best.value, list(ms)
