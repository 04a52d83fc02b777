"""Seeded synthetic workloads for the batched band solvers.

This module only *draws* inputs: random coefficients, manufactured right-hand
sides and the coefficient arrays of one ADI sweep of a nonlinear parabolic PDE.
It holds none of the solvers' arithmetic, so both the device path and the CPU
oracle may take their inputs from it.

Conventions
-----------
* Row i of a pentadiagonal (PD) system:
  e_i x_{i-2} + c_i x_{i-1} + d_i x_i + a_i x_{i+1} + b_i x_{i+2} = y_i;
  a tridiagonal (TD) system has e = b = 0.  Corner slots (e_0, e_1, c_0,
  a_{n-1}, b_{n-2}, b_{n-1}) are set to 0 here and are never read by a solver.
* Generators return dicts of float64 numpy arrays in *system-contiguous*
  layout [batch, n]; `interleave` converts to the device layout [n, ld]
  (element (row i, system s) at [i, s]).
* Seeds: configuration k uses numpy PCG64 with seed 1804 + k unless told
  otherwise.
"""
import math

import numpy as np

BASE_SEED = 1804
DIAG_NAMES = ("e", "c", "d", "a", "b")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def corner_mask(n):
    """Boolean masks (e, c, a, b) of the slots that lie inside the matrix."""
    i = np.arange(n)
    return (i >= 2), (i >= 1), (i <= n - 2), (i <= n - 3)


def band_matvec(diags, x):
    """y = A x for [batch, n] diagonals (used only to manufacture rhs)."""
    e, c, d, a, b = (diags[k] for k in DIAG_NAMES)
    y = d * x
    y[:, 1:] += c[:, 1:] * x[:, :-1]
    y[:, 2:] += e[:, 2:] * x[:, :-2]
    y[:, :-1] += a[:, :-1] * x[:, 1:]
    y[:, :-2] += b[:, :-2] * x[:, 2:]
    return y


def dominant_batch(batch, n, kind=5, seed=BASE_SEED, lo=-1.0, hi=1.0):
    """Random diagonally dominant PD (kind=5) or TD (kind=3) batch.

    Off-diagonals ~ U[lo, hi]; d = sum |off-diagonals in the row| + U[1, 2];
    x_true ~ U[-1, 1]; y = A x_true (manufactured right-hand side)."""
    rng = _rng(seed)
    me, mc, ma, mb = corner_mask(n)
    e = rng.uniform(lo, hi, (batch, n)) * me
    c = rng.uniform(lo, hi, (batch, n)) * mc
    a = rng.uniform(lo, hi, (batch, n)) * ma
    b = rng.uniform(lo, hi, (batch, n)) * mb
    if kind == 3:
        e[:] = 0.0
        b[:] = 0.0
    d = np.abs(e) + np.abs(c) + np.abs(a) + np.abs(b) + rng.uniform(1.0, 2.0, (batch, n))
    x_true = rng.uniform(-1.0, 1.0, (batch, n))
    out = dict(e=e, c=c, d=d, a=a, b=b, x_true=x_true)
    out["y"] = band_matvec(out, x_true)
    return out


def config0(kind, seed=BASE_SEED):
    """64 PD or 64 TD dominant systems, n = 1024."""
    return dominant_batch(64, 1024, kind=kind, seed=seed + (0 if kind == 5 else 1))


# --------------------------------------------------------------- PDE / ADI ---
def k_of_u(u):
    """Nonlinear coefficient k(u) = 1 + u^2."""
    return 1.0 + u * u


def smooth_field(N, seed, modes=4):
    """u0(x, y) = sum_{p,q<modes} a_pq cos(p pi x) cos(q pi y) on the nodes
    x_i = i h, h = 1/(N-1); a_pq ~ U[-1,1] 2^{-(p+q)}, scaled to max|u0| = 1."""
    rng = _rng(seed)
    amp = rng.uniform(-1.0, 1.0, (modes, modes))
    p = np.arange(modes)
    amp = amp * 2.0 ** (-(p[:, None] + p[None, :]))
    xs = np.linspace(0.0, 1.0, N)
    cx = np.cos(np.pi * p[:, None] * xs[None, :])  # [modes, N]
    u = cx.T @ amp @ cx                              # [N(y), N(x)]
    return u / np.abs(u).max()


def smooth_lines(nsys, n, seed, modes=4):
    """nsys independent smooth 1-D fields on n nodes (rows of [nsys, n])."""
    rng = _rng(seed)
    amp = rng.uniform(-1.0, 1.0, (nsys, modes)) * 2.0 ** (-np.arange(modes))
    xs = np.linspace(0.0, 1.0, n)
    u = amp @ np.cos(np.pi * np.arange(modes)[:, None] * xs[None, :])
    return u / np.abs(u).max(axis=1, keepdims=True)


def sweep_lines(v, r, order):
    """Coefficients of one implicit sweep  (I - tau L(k(v))) w = v  along the
    last axis of v ([nsys, n], one line per row), with r = tau / h^2:
      c_i = -r k_{i-1/2},  a_i = -r k_{i+1/2},  d_i = 1 + r (k_{i-1/2} + k_{i+1/2}),
      k_{i+-1/2} = (k(v_i) + k(v_{i+-1})) / 2,  rhs_i = v_i
    for interior rows, and zero-flux boundary rows with rhs 0:
      order 1 (TD):  [1, -1] at row 0 and [-1, 1] at row n-1;
      order 2 (PD):  [-3, 4, -1] at row 0 and [1, -4, 3] at row n-1
    (one-sided second-order derivative, not diagonally dominant)."""
    nsys, n = v.shape
    kv = k_of_u(v)
    kh = 0.5 * (kv[:, :-1] + kv[:, 1:])          # k_{i+1/2}, i = 0..n-2
    z = np.zeros((nsys, n))
    e, c, d, a, b, y = z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), z.copy()
    c[:, 1:-1] = -r * kh[:, :-1]
    a[:, 1:-1] = -r * kh[:, 1:]
    d[:, 1:-1] = 1.0 + r * (kh[:, :-1] + kh[:, 1:])
    y[:, 1:-1] = v[:, 1:-1]
    if order == 1:
        d[:, 0], a[:, 0] = 1.0, -1.0
        c[:, -1], d[:, -1] = -1.0, 1.0
    elif order == 2:
        d[:, 0], a[:, 0], b[:, 0] = -3.0, 4.0, -1.0
        e[:, -1], c[:, -1], d[:, -1] = 1.0, -4.0, 3.0
    else:
        raise ValueError("order must be 1 or 2")
    return dict(e=e, c=c, d=d, a=a, b=b, y=y)


def sweep_lines_interleaved(vt, r, order):
    """sweep_lines for lines stored along the FIRST axis (vt[i, s] = node i of
    line s, the batch-interleaved layout) on numpy arrays or torch tensors of
    any device: the same elementwise operations in the same order, so the
    coefficients are bitwise those of sweep_lines on vt.T (no fused
    multiply-add: every product and sum is its own rounded operation)."""
    n = vt.shape[0]
    kv = 1.0 + vt * vt
    kh = 0.5 * (kv[:-1] + kv[1:])               # k_{i+1/2}, i = 0..n-2
    zeros = (lambda: vt * 0.0)
    e, c, d, a, b, y = zeros(), zeros(), zeros(), zeros(), zeros(), zeros()
    c[1:-1] = -r * kh[:-1]
    a[1:-1] = -r * kh[1:]
    d[1:-1] = 1.0 + r * (kh[:-1] + kh[1:])
    y[1:-1] = vt[1:-1]
    if order == 1:
        d[0], a[0] = 1.0, -1.0
        c[-1], d[-1] = -1.0, 1.0
    elif order == 2:
        d[0], a[0], b[0] = -3.0, 4.0, -1.0
        e[-1], c[-1], d[-1] = 1.0, -4.0, 3.0
    else:
        raise ValueError("order must be 1 or 2")
    return dict(e=e, c=c, d=d, a=a, b=b, y=y)


def adi_sweep(u, r, order, axis):
    """Systems of one sweep of a 2-D field u[iy, ix]: axis='x' gives one
    system per grid row (lines along x), axis='y' one per grid column."""
    lines = u if axis == "x" else u.T
    return sweep_lines(np.ascontiguousarray(lines), r, order)


def config1(r=4.0, N=2048, seed=BASE_SEED + 1):
    """First y-sweep of the ADI step on an N x N grid: N PD systems
    (second-order boundary rows) and N TD systems (first-order), n = N."""
    u0 = smooth_field(N, seed)
    return adi_sweep(u0, r, 2, "y"), adi_sweep(u0, r, 1, "y"), u0


def config2_sizes(count=10000, lo=64, hi=65536, seed=BASE_SEED + 2):
    """System sizes n = floor(exp(U[ln lo, ln hi])) (log-uniform)."""
    rng = _rng(seed)
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(np.int64)


def dominant_groups(slot_sizes, seed=BASE_SEED + 2, device="cuda"):
    """Diagonally dominant PD systems (off-diagonals U[-1,1], d = sum|off| +
    U[1,2], x_true ~ U[-1,1], y = A x_true) in groups of 16: slot_sizes[16 g + l]
    is the length of the system in lane l of group g (0 = empty); group g is
    an [n_g][16] block (n_g = max of its lanes) and the blocks follow each
    other.  Generated on `device` with a seeded torch generator; returns flat
    float64 tensors e, c, d, a, b, y, x_true (positions of no system and slots
    outside a matrix hold 0)."""
    import torch
    sn = torch.as_tensor(np.asarray(slot_sizes, dtype=np.int64), device=device)
    groups = sn.numel() // 16
    gn = sn.view(groups, 16).max(dim=1).values
    elems = int(gn.sum()) * 16
    gid = torch.repeat_interleave(torch.arange(groups, device=device), gn * 16)
    goff = torch.cumsum(gn * 16, 0) - gn * 16
    pos = torch.arange(elems, device=device)
    row = (pos - goff[gid]) // 16
    nl = sn[gid * 16 + pos % 16]
    inside = row < nl
    masks = {"e": inside & (row >= 2), "c": inside & (row >= 1),
             "a": inside & (row <= nl - 2), "b": inside & (row <= nl - 3)}
    gen = torch.Generator(device=device).manual_seed(int(seed))

    def uni(lo, hi):
        return torch.rand(elems, generator=gen, device=device, dtype=torch.float64) * (hi - lo) + lo
    out = {}
    offsum = torch.zeros(elems, device=device, dtype=torch.float64)
    for k in ("e", "c", "a", "b"):
        out[k] = uni(-1.0, 1.0) * masks[k]
        offsum += out[k].abs()
    out["d"] = (offsum + uni(1.0, 2.0)) * inside
    x = uni(-1.0, 1.0) * inside
    y = out["d"] * x
    y[32:] += out["e"][32:] * x[:-32]
    y[16:] += out["c"][16:] * x[:-16]
    y[:-16] += out["a"][:-16] * x[16:]
    y[:-32] += out["b"][:-32] * x[32:]
    out["y"], out["x_true"] = y, x
    return out


def config3(nsys=256, n=1_000_000, r=4.0, seed=BASE_SEED + 3):
    """nsys PD lines of length n from smooth 1-D fields (second-order rows)."""
    return sweep_lines(smooth_lines(nsys, n, seed), r, 2)


# ----------------------------------------------------------------- layout ---
def padded_ld(batch, align=64):
    return ((batch + align - 1) // align) * align


def interleave(arr, ld=None, fill=0.0):
    """[batch, n] system-contiguous -> [n, ld] batch-interleaved."""
    arr = np.asarray(arr, dtype=np.float64)
    batch, n = arr.shape
    ld = padded_ld(batch) if ld is None else ld
    out = np.full((n, ld), fill, dtype=np.float64)
    out[:, :batch] = arr.T
    return out


def deinterleave(arr, batch):
    """[n, ld] batch-interleaved -> [batch, n] system-contiguous."""
    return np.ascontiguousarray(np.asarray(arr)[:, :batch].T)
