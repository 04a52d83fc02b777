"""Learned start vector for the Stone method (include/warmstart.h).

Binding of the warm-start part of libbandsolve (argument marshalling only:
features, network, loss, Adam and the start vector all run in its kernels),
plus the loop that trains the network on solutions of earlier ADI sweeps
and uses it.

Algorithm 1 of Veneva & Ayriyan (arXiv:1804.09666, Sec. 2) starts from a
free x^(0); with Hotelling-Bodewig steps in place of the triangular solves
the iteration count falls with ||b - A x^(0)||, which is what a good start
vector buys.  The network maps one 64-row patch of a system -- its five
diagonals, right-hand side and previous-step solution -- to the patch of
x^(0) - u_prev.
"""
import ctypes
import math

import numpy as np
import torch

from . import bandsolve as bs
from . import workloads as wl

WS_F32, WS_BF16 = 1, 2
OP_FORWARD, OP_TRAIN = 0, 1
PATCH, NFEAT, IN, HIDDEN, OUT = 64, 7, 448, 256, 64
EXPORTED = ("ws_param_count", "ws_workspace_bytes", "ws_gemm_nt", "ws_convert", "ws_forward",
            "ws_infer", "ws_backward", "ws_mse", "ws_adam", "ws_features", "ws_apply", "ws_predict")
TORCH_DTYPE = {WS_F32: torch.float32, WS_BF16: torch.bfloat16}

_lib = None


def load():
    """The warm-start entry points of libbandsolve.so.  No fallback."""
    global _lib
    if _lib is not None:
        return _lib
    lib = bs.load()
    i32, i64, vp, sz, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_float
    sig = {
        "ws_param_count": (i64, []),
        "ws_workspace_bytes": (sz, [i32, i32, i64]),
        "ws_gemm_nt": (i32, [i32, i64, i64, i64, vp, vp, vp, i32, vp, vp, vp, vp]),
        "ws_convert": (i32, [i32, i64, vp, vp, vp]),
        "ws_forward": (i32, [i32, i64, vp, vp, vp, vp, vp, sz, vp]),
        "ws_infer": (i32, [i64, vp, vp, vp, vp, vp]),
        "ws_backward": (i32, [i32, i64, vp, vp, vp, vp, vp, vp, sz, vp]),
        "ws_mse": (i32, [i64, vp, vp, vp, vp, vp, vp]),
        "ws_adam": (i32, [i32, i64, vp, vp, vp, vp, vp, f32, f32, f32, f32, i32, vp]),
        "ws_features": (i32, [i32, i64, i64, i64, ctypes.c_void_p * 7, ctypes.c_float * 14, vp,
                              vp]),
        "ws_apply": (i32, [i64, i64, i64, vp, vp, f32, f32, vp, vp]),
        "ws_predict": (i32, [i64, i64, i64, ctypes.c_void_p * 7, ctypes.c_float * 14, vp, vp, f32,
                             f32, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _st(stream):
    return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def _ok(status, what):
    if status != bs.BS_OK:
        raise bs.BandSolveError(status, what)


def param_count():
    return int(load().ws_param_count())


def workspace(op, dtype, P, device="cuda"):
    nbytes = load().ws_workspace_bytes(op, dtype, P)
    if nbytes == ctypes.c_size_t(-1).value:
        raise bs.BandSolveError(bs.BS_EINVAL, "ws_workspace_bytes")
    return torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=device)


def gemm_nt(A, B, bias=None, relu=False, mask=None, out32=None, outT=None, stream=None):
    """C = A B^T (+ bias, ReLU, mask) on the matrix cores; A [M, K], B [N, K]
    in float32 or bfloat16."""
    dtype = WS_BF16 if A.dtype == torch.bfloat16 else WS_F32
    M, K = A.shape
    N = B.shape[0]
    _ok(load().ws_gemm_nt(dtype, M, N, K, _p(A), _p(B), _p(bias), int(relu), _p(mask),
                          _p(out32), _p(outT), _st(stream)), "ws_gemm_nt")
    return out32 if out32 is not None else outT


def convert(x32, dtype, out=None, stream=None):
    out = torch.empty(x32.shape, dtype=TORCH_DTYPE[dtype], device=x32.device) if out is None else out
    _ok(load().ws_convert(dtype, x32.numel(), _p(x32), _p(out), _st(stream)), "ws_convert")
    return out


def forward(dtype, X, p32, pT, Y=None, ws=None, stream=None):
    P = X.shape[0]
    Y = torch.empty((P, OUT), dtype=torch.float32, device=X.device) if Y is None else Y
    ws = workspace(OP_FORWARD, dtype, P, X.device) if ws is None else ws
    _ok(load().ws_forward(dtype, P, _p(X), _p(p32), _p(pT), _p(Y), _p(ws),
                          ws.numel() * ws.element_size(), _st(stream)), "ws_forward")
    return Y


def infer(X, p32, pT, Y=None, stream=None):
    """Y = network(X) for BF16 X and weights in one fused kernel (no workspace;
    the same result as forward(WS_BF16, ...))."""
    P = X.shape[0]
    Y = torch.empty((P, OUT), dtype=torch.float32, device=X.device) if Y is None else Y
    _ok(load().ws_infer(P, _p(X), _p(p32), _p(pT), _p(Y), _st(stream)), "ws_infer")
    return Y


def backward(dtype, X, p32, pT, dY, grads, ws, stream=None):
    P = X.shape[0]
    _ok(load().ws_backward(dtype, P, _p(X), _p(p32), _p(pT), _p(dY), _p(grads), _p(ws),
                           ws.numel() * ws.element_size(), _st(stream)), "ws_backward")
    return grads


def mse(Y, T, dY, loss, partial, stream=None):
    _ok(load().ws_mse(Y.shape[0], _p(Y), _p(T), _p(dY), _p(loss), _p(partial), _st(stream)),
        "ws_mse")
    return loss


def adam(dtype, p32, pT, grads, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _ok(load().ws_adam(dtype, p32.numel(), _p(p32), _p(pT), _p(grads), _p(m), _p(v), lr, beta1,
                       beta2, eps, int(step), _st(stream)), "ws_adam")


def features(dtype, planes, norm, n, batch, X=None, stream=None):
    """planes: 7 float64 device tensors [n, ld] (e, c, d, a, b, rhs, u_prev);
    norm: 14 floats (7 means, 7 scales)."""
    ld = planes[2].shape[1]
    P = batch * ((n + PATCH - 1) // PATCH)
    X = torch.empty((P, IN), dtype=TORCH_DTYPE[dtype], device=planes[2].device) if X is None else X
    lib = load()
    arr = (ctypes.c_void_p * 7)(*[t.data_ptr() for t in planes])
    nm = (ctypes.c_float * 14)(*[float(v) for v in norm])
    _ok(lib.ws_features(dtype, n, batch, ld, arr, nm, _p(X), _st(stream)), "ws_features")
    return X


def apply(Y, uprev, mu_t, sigma_t, n, batch, x0=None, stream=None):
    ld = uprev.shape[1]
    x0 = torch.empty_like(uprev) if x0 is None else x0
    _ok(load().ws_apply(n, batch, ld, _p(Y), _p(uprev), float(mu_t), float(sigma_t), _p(x0),
                        _st(stream)), "ws_apply")
    return x0


def predict_fused(planes, norm, p32, pT, mu_t, sigma_t, n, batch, x0=None, stream=None):
    """features -> BF16 network -> x0 in one kernel (ws_predict); bitwise
    apply(infer(features(WS_BF16, ...)))."""
    ld = planes[6].shape[1]
    x0 = torch.empty_like(planes[6]) if x0 is None else x0
    arr = (ctypes.c_void_p * 7)(*[t.data_ptr() for t in planes])
    nm = (ctypes.c_float * 14)(*[float(v) for v in norm])
    _ok(load().ws_predict(n, batch, ld, arr, nm, _p(p32), _p(pT), float(mu_t), float(sigma_t),
                          _p(x0), _st(stream)), "ws_predict")
    return x0


def init_params(seed=0):
    """Host-side initial parameters: W uniform in +-sqrt(6 / fan_in) (He),
    biases 0; returned as a float32 numpy vector in the ABI's layout."""
    rng = np.random.default_rng(seed)
    dims = (IN, HIDDEN, HIDDEN, HIDDEN, OUT)
    parts = []
    for k in range(4):
        lim = math.sqrt(6.0 / dims[k]) if k < 3 else math.sqrt(3.0 / dims[k])
        parts.append(rng.uniform(-lim, lim, dims[k + 1] * dims[k]))
        parts.append(np.zeros(dims[k + 1]))
    return np.concatenate(parts).astype(np.float32)


class WarmStart:
    """The network's parameters, Adam state and input/output scaling."""

    def __init__(self, dtype=WS_BF16, seed=0, device="cuda"):
        self.dtype = dtype
        self.device = device
        self.p32 = torch.from_numpy(init_params(seed)).to(device)
        self.pT = convert(self.p32, dtype) if dtype == WS_BF16 else self.p32
        self.m = torch.zeros_like(self.p32)
        self.v = torch.zeros_like(self.p32)
        self.grads = torch.zeros_like(self.p32)
        self.step = 0
        self.norm = [0.0] * 7 + [1.0] * 7
        self.mu_t, self.sigma_t = 0.0, 1.0
        self._train = {}

    def train_step(self, X, T, lr):
        """One Adam step on the minibatch (X [P, 448] in the compute dtype,
        T [P, 64] FP32 scaled targets); returns the loss as a device tensor."""
        P = X.shape[0]
        st = self._train.get(P)
        if st is None:
            st = dict(ws=workspace(OP_TRAIN, self.dtype, P, self.device),
                      Y=torch.empty((P, OUT), dtype=torch.float32, device=self.device),
                      dY=torch.empty((P, OUT), dtype=torch.float32, device=self.device),
                      loss=torch.zeros(1, dtype=torch.float64, device=self.device),
                      part=torch.empty(P // 4 + 1, dtype=torch.float64, device=self.device))
            self._train[P] = st
        forward(self.dtype, X, self.p32, self.pT, st["Y"], st["ws"])
        mse(st["Y"], T, st["dY"], st["loss"], st["part"])
        backward(self.dtype, X, self.p32, self.pT, st["dY"], self.grads, st["ws"])
        self.step += 1
        adam(self.dtype, self.p32, self.pT if self.dtype == WS_BF16 else None, self.grads,
             self.m, self.v, lr, self.step)
        return st["loss"]

    def save(self, path):
        """Checkpoint: parameters, Adam moments and step, and the input/output
        scaling, as one .npz (plain arrays; nothing executable)."""
        np.savez(path, p32=self.p32.cpu().numpy(), m=self.m.cpu().numpy(),
                 v=self.v.cpu().numpy(), step=np.int64(self.step), dtype=np.int32(self.dtype),
                 norm=np.asarray(self.norm, dtype=np.float64),
                 target=np.asarray([self.mu_t, self.sigma_t], dtype=np.float64))

    @classmethod
    def restore(cls, path, device="cuda"):
        """A WarmStart from save(); training continues where it stopped."""
        with np.load(path, allow_pickle=False) as z:
            net = cls(int(z["dtype"]), device=device)
            net.p32.copy_(torch.from_numpy(z["p32"]))
            net.m.copy_(torch.from_numpy(z["m"]))
            net.v.copy_(torch.from_numpy(z["v"]))
            net.step = int(z["step"])
            net.norm = [float(x) for x in z["norm"]]
            net.mu_t, net.sigma_t = (float(x) for x in z["target"])
        if net.dtype == WS_BF16:
            convert(net.p32, net.dtype, out=net.pT)
        return net

    def fit_scaling(self, samples, n, batch):
        """Feature means and scales and the target scaling from training
        sweeps: samples = [(planes, solution), ...] as adi_trajectory hands
        them out."""
        unit = [0.0] * 7 + [1.0] * 7
        raw = torch.cat([features(WS_F32, planes, unit, n, batch) for planes, _ in samples])
        raw = raw.view(raw.shape[0], NFEAT, PATCH).transpose(0, 1).reshape(NFEAT, -1)
        mean = raw.double().mean(dim=1)
        std = raw.double().std(dim=1).clamp_min(1e-30)
        self.norm = [float(v) for v in mean.cpu()] + [float(v) for v in std.cpu()]
        t = torch.cat([(w - planes[6])[:, :batch].flatten() for planes, w in samples])
        self.mu_t = float(t.mean())
        self.sigma_t = max(float(t.std()), 1e-30)

    def targets(self, planes, w, n, batch):
        """Scaled training targets (w - u_prev - mu_t) / sigma_t in patch
        layout (FP32 [P, 64]), gathered by the feature kernel: with u_prev = 0
        its residual feature is the plane itself."""
        zero = torch.zeros_like(w)
        tp = list(planes[:5]) + [w - planes[6], zero]
        nt = [0.0] * 7 + [1.0] * 7
        nt[5], nt[12] = self.mu_t, self.sigma_t
        return features(WS_F32, tp, nt, n, batch)[:, 5 * PATCH:6 * PATCH].contiguous()

    def predict(self, diags, rhs, uprev, n, batch, x0=None, ws=None, X=None, Y=None):
        """x0 for a batch of pentadiagonal systems (device [n, ld] float64)."""
        planes = list(diags) + [rhs, uprev]
        if self.dtype == WS_BF16:   # one fused launch
            return predict_fused(planes, self.norm, self.p32, self.pT, self.mu_t, self.sigma_t,
                                 n, batch, x0)
        X = features(self.dtype, planes, self.norm, n, batch, X)
        Y = forward(self.dtype, X, self.p32, self.pT, Y, ws)
        return apply(Y, uprev, self.mu_t, self.sigma_t, n, batch, x0)


# --------------------------------------------------------------- the PDE ---
def adi_steps(N, r=4.0, seed=wl.BASE_SEED + 4, device="cuda"):
    """Endless time steps of u_t = (k(u)u_x)_x + (k(u)u_y)_y, k = 1 + u^2, on
    an N x N grid (locally one-dimensional ADI: an x-sweep, then a y-sweep,
    each with the second-order boundary rows), every sweep solved by
    band_solve.  Yields (step, planes, w) for each x-sweep: the batch-
    interleaved [N, N] device planes (e, c, d, a, b, rhs, u_prev) -- u_prev
    the previous step's x-sweep solution (the field itself at step 0) -- and
    the sweep's solution w."""
    u = torch.from_numpy(wl.smooth_field(N, seed)).to(device)   # [y, x]
    w_prev = None
    info = torch.empty(N, dtype=torch.int32, device=device)
    step = 0
    while True:
        vt = bs.pack_interleave(u)                               # x-lines: [x, y]
        sw = wl.sweep_lines_interleaved(vt, r, 2)
        diags = [sw[k] for k in ("e", "c", "d", "a", "b")]
        w, _ = bs.solve(diags, sw["y"], kind=5, batch=N, info=info)
        yield step, diags + [sw["y"], w_prev if w_prev is not None else vt], w
        w_prev = w
        sy = wl.sweep_lines_interleaved(bs.pack_interleave(w), r, 2)   # y-lines: [y, x]
        u, _ = bs.solve([sy[k] for k in ("e", "c", "d", "a", "b")], sy["y"], kind=5, batch=N,
                        info=info)
        step += 1


def adi_trajectory(N, steps, r=4.0, seed=wl.BASE_SEED + 4, device="cuda", on_xsweep=None):
    """Runs `steps` steps of adi_steps, calling on_xsweep(step, planes, w)."""
    for step, planes, w in adi_steps(N, r, seed, device):
        if step >= steps:
            break
        if on_xsweep is not None:
            on_xsweep(step, planes, w)
