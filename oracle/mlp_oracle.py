"""FP64 CPU oracle for the learned SIP warm start (TEST INFRASTRUCTURE).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use this module; the product never imports it, and it imports
nothing of the product.  Plain numpy in float64, written from the definitions:

  * patch features: system s, rows [64 j, 64 j + 64) give one input vector of
    7 x 64 values -- the diagonals e, c, d, a, b, the residual of the
    previous-step solution r0 = rhs - A u_prev (the right-hand side enters
    through it) and u_prev itself, each standardised with a per-feature mean
    and scale; slots outside the matrix (e_0, e_1, c_0, a_{n-1}, b_{n-2},
    b_{n-1}) count as raw value 0 before scaling, and rows past n are 0 after
    it;
  * the network: three hidden layers with ReLU and a linear output,
        h1 = relu(X W1^T + b1), h2 = relu(h1 W2^T + b2),
        h3 = relu(h2 W3^T + b3), Y = h3 W4^T + b4;
  * the loss: mean squared error over all outputs, and its gradient by the
    chain rule (backward pass written out layer by layer);
  * Adam (Kingma & Ba 2015, Algorithm 1) with bias-corrected moments;
  * the start vector: x0 = u_prev + mu_t + sigma_t Y for the rows of each
    patch that lie inside the system.

The SIP iteration these start vectors feed is Algorithm 1 of Veneva & Ayriyan
(arXiv:1804.09666, Sec. 2); its x^(0) is free, which is what the network
predicts.  `bf16=True` rounds every GEMM operand (inputs, weights, stored
activations and the stored output gradient) to bfloat16 first, as the
mixed-precision kernels store them; arithmetic stays float64.
"""
import numpy as np

PATCH = 64
NFEAT = 7
DIMS = (NFEAT * PATCH, 256, 256, 256, PATCH)  # in, hidden x 3, out


# ------------------------------------------------------------------ bf16 ---
def bf16_round(x):
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64: bfloat16 keeps the top 16 bits of the float32 pattern."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


# ------------------------------------------------------------- parameters --
def param_shapes(dims=DIMS):
    """[(W1, b1), ...]: W_k is [out, in] (row-major), b_k is [out]."""
    return [((dims[k + 1], dims[k]), (dims[k + 1],)) for k in range(len(dims) - 1)]


def unpack(flat, dims=DIMS):
    """Flat parameter vector (W1, b1, W2, b2, ...) -> list of (W, b)."""
    out, o = [], 0
    for ws, bs_ in param_shapes(dims):
        nw = ws[0] * ws[1]
        out.append((flat[o:o + nw].reshape(ws), flat[o + nw:o + nw + bs_[0]]))
        o += nw + bs_[0]
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def param_count(dims=DIMS):
    return sum(a[0] * a[1] + b[0] for a, b in param_shapes(dims))


# --------------------------------------------------------------- features --
def features(e, c, d, a, b, rhs, uprev, mean, scale):
    """[batch, n] system-contiguous arrays -> X [batch * ceil(n/64), 448];
    patch index p = s * ceil(n/64) + j."""
    batch, n = d.shape
    npatch = -(-n // PATCH)
    raw = [np.array(v, dtype=np.float64, copy=True) for v in (e, c, d, a, b, rhs, uprev)]
    # slots outside the matrix count as 0
    raw[0][:, :2] = 0.0
    raw[1][:, :1] = 0.0
    raw[3][:, n - 1:] = 0.0
    raw[4][:, max(n - 2, 0):] = 0.0
    # r0_i = rhs_i - (((d_i u_i + e_i u_{i-2}) + c_i u_{i-1}) + a_i u_{i+1}) + b_i u_{i+2},
    # terms outside the matrix omitted
    u = raw[6]
    ax = raw[2] * u
    ax[:, 2:] = ax[:, 2:] + raw[0][:, 2:] * u[:, :-2]
    ax[:, 1:] = ax[:, 1:] + raw[1][:, 1:] * u[:, :-1]
    ax[:, :-1] = ax[:, :-1] + raw[3][:, :-1] * u[:, 1:]
    ax[:, :-2] = ax[:, :-2] + raw[4][:, :-2] * u[:, 2:]
    raw[5] = raw[5] - ax
    X = np.zeros((batch * npatch, NFEAT * PATCH))
    for f in range(NFEAT):
        z = (raw[f] - mean[f]) / scale[f]
        zp = np.zeros((batch, npatch * PATCH))
        zp[:, :n] = z
        X[:, f * PATCH:(f + 1) * PATCH] = zp.reshape(batch * npatch, PATCH)
    return X


def apply_start(Y, uprev, mu_t, sigma_t):
    """Y [batch * ceil(n/64), 64] -> x0 [batch, n] = u_prev + mu_t + sigma_t Y."""
    batch, n = uprev.shape
    npatch = -(-n // PATCH)
    y = Y.reshape(batch, npatch * PATCH)[:, :n]
    return uprev + (mu_t + sigma_t * y)


# ----------------------------------------------------------------- network --
def forward(X, flat, dims=DIMS, bf16=False):
    """Returns (Y, activations) with activations = [X, h1, h2, h3] as the
    backward pass reads them (bf16-rounded when bf16=True)."""
    rnd = bf16_round if bf16 else (lambda v: v)
    layers = unpack(np.asarray(flat, dtype=np.float64), dims)
    acts = [rnd(X)]
    h = acts[0]
    for k, (W, b) in enumerate(layers):
        z = h @ rnd(W).T + b
        if k < len(layers) - 1:
            h = rnd(np.maximum(z, 0.0))
            acts.append(h)
        else:
            h = z
    return h, acts


def mse(Y, T):
    """Loss = mean((Y - T)^2) and dL/dY."""
    diff = Y - T
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


def backward(dY, acts, flat, dims=DIMS, bf16=False):
    """Gradient of the loss w.r.t. the flat parameter vector, given dL/dY
    and the activations of forward().  Output layer: db = sum_rows(dY),
    dW = dY^T h; hidden layers: g = (g_next W_next) * [h > 0], db = sum_rows(g),
    dW = g^T h_in.  With bf16=True every GEMM operand is bf16-rounded (dY as
    GEMM operand; each hidden g as it is stored), sums read the stored g."""
    rnd = bf16_round if bf16 else (lambda v: v)
    layers = unpack(np.asarray(flat, dtype=np.float64), dims)
    L = len(layers)
    grads = [None] * L
    g_sum = np.asarray(dY, dtype=np.float64)  # what the bias sum reads
    g_op = rnd(g_sum)                          # what the GEMMs read
    for k in range(L - 1, -1, -1):
        grads[k] = (g_op.T @ acts[k], np.sum(g_sum, axis=0))
        if k > 0:
            W, _ = layers[k]
            g_sum = rnd((g_op @ rnd(W)) * (acts[k] > 0))
            g_op = g_sum
    return pack(grads)


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
