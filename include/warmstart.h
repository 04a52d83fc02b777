/* warmstart.h -- C ABI of the learned start vector for the Stone method
 * (SIP), part of libbandsolve (gfx950).
 *
 * Algorithm 1 of Veneva & Ayriyan (arXiv:1804.09666, Sec. 2) iterates from a
 * free start vector x^(0); the number of steps to a tolerance falls as
 * x^(0) nears the solution.  This part predicts x^(0) for the systems of an
 * ADI sweep with a small network trained on solutions of earlier sweeps:
 *
 *   features  system s, rows [64 j, 64 j + 64) ("patch" p = s * P_n + j,
 *             P_n = ceil(n / 64)) give one input row of 448 values (7 blocks
 *             of 64): the diagonals e, c, d, a, b, the residual of the
 *             previous-step solution r0 = rhs - A u_prev (through which the
 *             right-hand side enters: a BF16 copy of rhs and u_prev could not
 *             resolve their difference) and u_prev, each standardised as
 *             (v - mean_f) / scale_f.  Slots outside the matrix (e_0, e_1,
 *             c_0, a_{n-1}, b_{n-2}, b_{n-1}) count as 0 before scaling; rows
 *             past n are 0 after it.
 *   network   448 -> 256 -> 256 -> 256 -> 64, ReLU after each hidden layer:
 *             h1 = relu(X W1^T + b1), h2 = relu(h1 W2^T + b2),
 *             h3 = relu(h2 W3^T + b3), Y = h3 W4^T + b4.
 *   start     x0 = u_prev + mu_t + sigma_t * Y for the rows of the patch
 *             inside the system.
 *
 * Parameters are one flat FP32 vector, per layer k = 1..4: W_k (row-major
 * [out, in]) then b_k ([out]); ws_param_count() elements.  Compute precision
 * WS_BF16 multiplies BF16 copies of inputs, weights and stored activations on
 * the matrix cores with FP32 accumulation (the BF16 copy of the parameters is
 * the same layout in bfloat16; biases are always read from the FP32 vector);
 * WS_F32 does the same in FP32.
 *
 * All pointers are device pointers owned by the caller; nothing is allocated.
 * Calls enqueue on `stream` (hipStream_t as void*, NULL = default) and
 * return a bs_status (bandsolve.h): BS_EINVAL for bad sizes, NULL or
 * misaligned pointers (every array 16-byte aligned), BS_EWORKSPACE for a
 * short workspace, BS_ELAUNCH for a failed launch.
 */
#ifndef WARMSTART_H
#define WARMSTART_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ws_dims_code { WS_PATCH = 64, WS_NFEAT = 7, WS_IN = 448, WS_HIDDEN = 256, WS_OUT = 64 };
enum ws_dtype_code { WS_F32 = 1, WS_BF16 = 2 };
enum ws_op_code { WS_OP_FORWARD = 0, WS_OP_TRAIN = 1 };

/* Number of FP32 parameters (weights and biases of the four layers). */
int64_t ws_param_count(void);

/* Workspace bytes for `op` on P patches: WS_OP_FORWARD keeps the three
 * hidden activations; WS_OP_TRAIN also the backward pass's buffers (the
 * backward pass reads the activations its ws_forward call left there).
 * (size_t)-1 for invalid arguments. */
size_t ws_workspace_bytes(int32_t op, int32_t dtype, int64_t P);

/* C[M,N] = A[M,K] B[N,K]^T (row-major, K contiguous) with FP32 accumulation,
 * then + bias[n] (FP32, nullable), ReLU if relu != 0, times [mask[m,n] > 0]
 * (dtype array, nullable); written to C32 (FP32, nullable) and/or CT (dtype,
 * nullable), both row-major [M, N].  K must be a multiple of 8 (BF16) or 4
 * (FP32).  The matrix-core kernel the network runs on, exported for tests. */
int32_t ws_gemm_nt(int32_t dtype, int64_t M, int64_t N, int64_t K, const void* A,
                   const void* B, const float* bias, int32_t relu, const void* mask,
                   float* C32, void* CT, void* stream);

/* FP32 -> dtype copy of `count` elements (the BF16 copy of the parameters). */
int32_t ws_convert(int32_t dtype, int64_t count, const float* in, void* out, void* stream);

/* Y[P, 64] (FP32) = network(X[P, 448]) with X and weights in dtype.
 * params32: FP32 parameters (biases), paramsT: the dtype copy (weights;
 * may equal params32 for WS_F32). */
int32_t ws_forward(int32_t dtype, int64_t P, const void* X, const float* params32,
                   const void* paramsT, float* Y, void* workspace, size_t ws_bytes,
                   void* stream);

/* Inference only, BF16 (X and paramsT in bfloat16): Y[P, 64] (FP32) =
 * network(X[P, 448]) with one kernel that carries each tile of patches
 * through all four layers (activations in LDS, weights read from L2), so no
 * activation goes to memory and no workspace is needed.  The rounding points
 * and the order of the FP32 accumulations are those of ws_forward with
 * WS_BF16, whose result it reproduces.  All pointers 16-byte aligned. */
int32_t ws_infer(int64_t P, const void* X, const float* params32, const void* paramsT, float* Y,
                 void* stream);

/* Gradient of a loss w.r.t. the parameters (FP32, ws_param_count()
 * elements, overwritten) given dL/dY (FP32 [P, 64]), after ws_forward on the
 * same X, parameters and workspace (WS_OP_TRAIN size).  P must be a multiple
 * of 8. */
int32_t ws_backward(int32_t dtype, int64_t P, const void* X, const float* params32,
                    const void* paramsT, const float* dY, float* grads, void* workspace,
                    size_t ws_bytes, void* stream);

/* Mean squared error over P*64 outputs: dY = 2 (Y - T) / (P*64) and
 * *loss (device double) = mean((Y - T)^2).  partial: ceil(P/4) doubles of
 * scratch. */
int32_t ws_mse(int64_t P, const float* Y, const float* T, float* dY, double* loss,
               double* partial, void* stream);

/* One Adam step (Kingma & Ba 2015) on `count` parameters, step >= 1:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps);
 * and pT = dtype copy of the new p (nullable). */
int32_t ws_adam(int32_t dtype, int64_t count, float* params, void* paramsT,
                const float* grads, float* m, float* v, float lr, float beta1, float beta2,
                float eps, int32_t step, void* stream);

/* Patch features of a batch of pentadiagonal systems: planes[0..6] =
 * e, c, d, a, b, rhs, u_prev (FP64, batch-interleaved [n, ld]); norm[0..6] =
 * means, norm[7..13] = scales (host array) of the seven features (feature 5
 * is the residual rhs - A u_prev).  X: [batch * ceil(n/64), 448] in dtype. */
int32_t ws_features(int32_t dtype, int64_t n, int64_t batch, int64_t ld,
                    const double* const planes[7], const float norm[14], void* X,
                    void* stream);

/* x0[i*ld + s] = u_prev[i*ld + s] + mu_t + sigma_t * Y[p, i - 64 j] for the
 * rows i of every patch p = s * ceil(n/64) + j inside the system. */
int32_t ws_apply(int64_t n, int64_t batch, int64_t ld, const float* Y, const double* uprev,
                 float mu_t, float sigma_t, double* x0, void* stream);

/* features -> network (BF16, as ws_infer) -> start vector in one launch:
 * the x0 that ws_apply gives for the Y of ws_infer on the X of
 * ws_features(WS_BF16, ...), bit for bit, without X or Y going through
 * memory.  planes, norm, mu_t, sigma_t as for ws_features / ws_apply
 * (planes[6] is u_prev); x0 [n, ld] may not alias a plane. */
int32_t ws_predict(int64_t n, int64_t batch, int64_t ld, const double* const planes[7],
                   const float norm[14], const float* params32, const void* paramsT,
                   float mu_t, float sigma_t, double* x0, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WARMSTART_H */
