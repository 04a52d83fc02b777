// mlp.hip -- the learned SIP start vector (declared in include/warmstart.h):
// patch features, a 448-256-256-256-64 ReLU network on the matrix cores
// (forward, backward, Adam), and the start vector x0.
//
// One GEMM kernel serves every product, C = A B^T with both operands K-
// contiguous (the layout of X W^T with W stored [out, in]); the backward pass
// brings its operands into that layout with a tiled transpose.  A block
// computes a tile of C with four waves (2 x 2), each owning TI x TJ MFMA
// 32 x 32 tiles; K advances in slices of 128 bytes per row, double-buffered
// through LDS (the next slice is fetched while the matrix cores work).  Lane layout
// of v_mfma_f32_32x32x16_bf16 / v_mfma_f32_32x32x2_f32 (checked on the
// device): lane l holds A row (l mod 32) and B column (l mod 32) at
// k = (l div 32) * KS/2 .. + KS/2 - 1; accumulator v of lane l is
// C[8 (v div 4) + 4 (l div 32) + (v mod 4)][l mod 32].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "bandsolve.h"
#include "warmstart.h"

namespace wsm {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

template <typename T>
struct Mfma;
template <>
struct Mfma<bf16> {
  static constexpr int KS = 16;  // k per instruction
  typedef bf16x8 Frag;           // 8 values per lane
  static __device__ inline f32x16 run(Frag a, Frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  static constexpr int KS = 2;
  typedef float Frag;
  static __device__ inline f32x16 run(Frag a, Frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};

typedef uint32_t Vec16 __attribute__((ext_vector_type(4)));  // one 16-byte chunk

// TI x TJ MFMA tiles of 32 x 32 per wave, 2 x 2 waves per block: a block
// computes a (64 TI) x (64 TJ) tile of C.  Large wave tiles keep the LDS
// traffic per matrix-core instruction low (each fragment read from LDS feeds
// TJ or TI instructions).
template <typename T, int TI, int TJ>
__global__ __launch_bounds__(kThreads) void gemm_nt_kernel(int64_t M, int64_t N, int64_t K,
                                                           const T* __restrict__ A,
                                                           const T* __restrict__ B,
                                                           const float* __restrict__ bias,
                                                           int relu, const T* __restrict__ mask,
                                                           float* __restrict__ C32,
                                                           T* __restrict__ CT) {
  typedef Mfma<T> MF;
  constexpr int WM = 32 * TI, WN = 32 * TJ;   // wave tile
  constexpr int BM = 2 * WM, BN = 2 * WN;     // block tile
  constexpr int VEC = 16 / sizeof(T);         // elements per 16-byte chunk
  constexpr int BK = 128 / sizeof(T);         // K per stage: 128 bytes of every row
  constexpr int LDR = BK + VEC;               // LDS row pitch: 16 bytes of padding
  constexpr int CPR = BK / VEC;               // chunks per tile row (8)
  constexpr int CPA = BM * CPR / kThreads;    // chunks per thread, A
  constexpr int CPB = BN * CPR / kThreads;    // chunks per thread, B
  static_assert(CPA >= 1 && CPB >= 1, "tile");
  // two stages: the next K slice is fetched into registers while the matrix
  // cores work on the current one, then stored to the other stage
  __shared__ __attribute__((aligned(16))) T sA[2][BM * LDR];
  __shared__ __attribute__((aligned(16))) T sB[2][BN * LDR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  // block -> (row tile, column tile): blocks go to the 8 XCDs round-robin, so
  // the column tiles of one row tile are placed consecutively on one XCD and
  // its A rows come from that XCD's L2 after the first read
  int64_t rt, ctile;
  {
    const int64_t nrow = (M + BM - 1) / BM, ncol = (N + BN - 1) / BN;
    const int64_t b = blockIdx.x;
    if (nrow % 8 == 0) {
      const int64_t xcd = b % 8, k = b / 8;
      rt = (k / ncol) * 8 + xcd;
      ctile = k % ncol;
    } else {
      rt = b / ncol;
      ctile = b % ncol;
    }
  }
  const int64_t m0 = rt * BM, n0 = ctile * BN;
  f32x16 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
  const int hi = lane >> 5, lo = lane & 31;

  Vec16 ra[CPA], rb[CPB];
  auto fetch = [&](int64_t k0) {  // zero outside the matrices; K % VEC == 0
#pragma unroll
    for (int q = 0; q < CPA; ++q) {
      const int c = tid + q * kThreads;
      const int r = c / CPR, kc = (c % CPR) * VEC;
      const int64_t k = k0 + kc;
      ra[q] = Vec16{0u, 0u, 0u, 0u};
      if (m0 + r < M && k < K) ra[q] = *reinterpret_cast<const Vec16*>(A + (m0 + r) * K + k);
    }
#pragma unroll
    for (int q = 0; q < CPB; ++q) {
      const int c = tid + q * kThreads;
      const int r = c / CPR, kc = (c % CPR) * VEC;
      const int64_t k = k0 + kc;
      rb[q] = Vec16{0u, 0u, 0u, 0u};
      if (n0 + r < N && k < K) rb[q] = *reinterpret_cast<const Vec16*>(B + (n0 + r) * K + k);
    }
  };
  auto stash = [&](int st) {
#pragma unroll
    for (int q = 0; q < CPA; ++q) {
      const int c = tid + q * kThreads;
      *reinterpret_cast<Vec16*>(&sA[st][(c / CPR) * LDR + (c % CPR) * VEC]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < CPB; ++q) {
      const int c = tid + q * kThreads;
      *reinterpret_cast<Vec16*>(&sB[st][(c / CPR) * LDR + (c % CPR) * VEC]) = rb[q];
    }
  };
  const int64_t nk = (K + BK - 1) / BK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int st = (int)(kt & 1);
    if (kt + 1 < nk) fetch((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += MF::KS) {
      typename MF::Frag fa[TI], fb[TJ];
      const int ko = kk + hi * (MF::KS / 2);
#pragma unroll
      for (int t = 0; t < TI; ++t)
        fa[t] = *reinterpret_cast<const typename MF::Frag*>(&sA[st][(wm + 32 * t + lo) * LDR + ko]);
#pragma unroll
      for (int t = 0; t < TJ; ++t)
        fb[t] = *reinterpret_cast<const typename MF::Frag*>(&sB[st][(wn + 32 * t + lo) * LDR + ko]);
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = MF::run(fa[i], fb[j], acc[i][j]);
    }
    if (kt + 1 < nk) stash(st ^ 1);
    __syncthreads();
  }

  // ---- epilogue: bias, ReLU, mask; consecutive lanes write consecutive n --
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int64_t col = n0 + wn + 32 * j + lo;
      if (col >= N) continue;
      const float bv = bias ? bias[col] : 0.0f;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * hi + (v & 3);
        if (row >= M) continue;
        float val = acc[i][j][v] + bv;
        if (relu) val = val > 0.0f ? val : 0.0f;
        if (mask && !((float)mask[row * N + col] > 0.0f)) val = 0.0f;
        if (C32) C32[row * N + col] = val;
        if (CT) CT[row * N + col] = (T)val;
      }
    }
}

// ---- the whole network for a tile of patches (inference) ------------------
// One block carries 32 RT patches through all four layers.  The layer input
// sits in LDS (bf16, [32 RT][kFLD]); each of the NW waves computes 32 CJ of
// the hidden output columns (RT x CJ MFMA tiles of 32 x 32) with its weight
// fragments read straight from global memory: the weights stay in every
// XCD's L2, and a wave fetches the fragments of four k-steps together (a
// whole 128-byte line of each of its weight rows) while the matrix cores work
// on the four before.  Then the block writes relu(acc + b) back over the
// input as bf16 and moves on; the last layer's 64 columns go to `out(row,
// col, y)` in FP32 (wave w takes row tiles w, w + NW, ...: it has read the
// tile's rows of the last hidden layer before it calls out for them).  The
// MFMAs of a tile accumulate k in the same order as gemm_nt_kernel, and the
// rounding points (bf16 activations, FP32 accumulation, bias then ReLU) are
// the same, so Y is the layered forward pass's.  Two waves per SIMD (NW = 8)
// and 128 patches per block measured 633 us on 262 144 patches of the
// 448-512-512-512-64 network against 832 us with one wave per SIMD and 96.
constexpr int kFRT = 4;              // row tiles of 32 patches per block
constexpr int kFR = 32 * kFRT;       // patches per block
constexpr int kFLD = (WS_IN > WS_HIDDEN ? WS_IN : WS_HIDDEN) + 8;  // LDS row pitch (bf16)
constexpr int kInferWaves = 8;       // two waves per SIMD (one per SIMD: 357 against 291 us)

// One hidden layer on the LDS tile: h = relu(in W^T + b) over K input
// columns, written back over the tile.  K is a compile-time constant so that
// the k loop unrolls completely: the two fragment buffers then stay in fixed
// registers and each wait covers only the loads it needs.
template <int NW, int K>
__device__ __attribute__((always_inline)) inline void hidden_layer(bf16* __restrict__ sH,
                                                                   const bf16* __restrict__ Wl,
                                                                   const float* __restrict__ bl) {
  constexpr int RT = kFRT;
  constexpr int CJ = WS_HIDDEN / 32 / NW;  // column tiles of 32 per wave
  static_assert(K % 64 == 0, "k in groups of four MFMA steps");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int hi = lane >> 5, lo = lane & 31;
  const int n0 = wave * 32 * CJ;
  f32x16 acc[RT][CJ];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CJ; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
  const bf16* wrow[CJ];
#pragma unroll
  for (int j = 0; j < CJ; ++j) wrow[j] = Wl + (int64_t)(n0 + 32 * j + lo) * K + hi * 8;
  // fragments of four k-steps (64 values of k) per buffer
  bf16x8 fb[2][4][CJ];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < CJ; ++j) fb[0][q][j] = *reinterpret_cast<const bf16x8*>(wrow[j] + 16 * q);
#pragma clang loop unroll(full)
  for (int g = 0; g < K / 64; ++g) {
    const int h = g & 1;
    const int k0 = 64 * g;
    if (k0 + 64 < K) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < CJ; ++j)
          fb[h ^ 1][q][j] = *reinterpret_cast<const bf16x8*>(wrow[j] + k0 + 64 + 16 * q);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 16 * q;
      bf16x8 fa[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i)
        fa[i] = *reinterpret_cast<const bf16x8*>(&sH[(32 * i + lo) * kFLD + k + hi * 8]);
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[h][q][j], acc[i][j], 0, 0, 0);
    }
  }
  __syncthreads();  // every wave has read the layer input
#pragma unroll
  for (int j = 0; j < CJ; ++j) {
    const int col = n0 + 32 * j + lo;
    const float bv = bl[col];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = 32 * i + 8 * (v >> 2) + 4 * hi + (v & 3);
        float val = acc[i][j][v] + bv;
        val = val > 0.0f ? val : 0.0f;
        sH[row * kFLD + col] = (bf16)val;
      }
  }
  __syncthreads();
}

template <int NW, typename Out>
__device__ inline void network_tile(bf16* __restrict__ sH, const bf16* __restrict__ W,
                                    const float* __restrict__ p32, Out&& out) {
  constexpr int RT = kFRT;
  static_assert((WS_HIDDEN / 32 / NW) * 32 * NW == WS_HIDDEN, "hidden columns split over the waves");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int hi = lane >> 5, lo = lane & 31;
  int64_t wo = 0;  // offset of this layer's W (then b) in the parameter vector
  hidden_layer<NW, WS_IN>(sH, W + wo, p32 + wo + (int64_t)WS_HIDDEN * WS_IN);
  wo += (int64_t)WS_HIDDEN * WS_IN + WS_HIDDEN;
#pragma unroll 1
  for (int layer = 1; layer < 3; ++layer) {
    hidden_layer<NW, WS_HIDDEN>(sH, W + wo, p32 + wo + (int64_t)WS_HIDDEN * WS_HIDDEN);
    wo += (int64_t)WS_HIDDEN * WS_HIDDEN + WS_HIDDEN;
  }
  // output layer: (32 RT) x 64; wave w takes row tiles w, w + NW, ... and both column tiles
  {
    const int K = WS_HIDDEN;
    const float* bl = p32 + wo + (int64_t)WS_OUT * K;
    const bf16* wr0 = W + wo + (int64_t)lo * K + hi * 8;
    const bf16* wr1 = wr0 + (int64_t)32 * K;
    for (int ti = wave; ti < RT; ti += NW) {
      f32x16 acc0, acc1;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc0[v] = acc1[v] = 0.0f;
#pragma unroll 4
      for (int k = 0; k < K; k += 16) {
        const bf16x8 fa = *reinterpret_cast<const bf16x8*>(&sH[(32 * ti + lo) * kFLD + k + hi * 8]);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, *reinterpret_cast<const bf16x8*>(wr0 + k),
                                                       acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, *reinterpret_cast<const bf16x8*>(wr1 + k),
                                                       acc1, 0, 0, 0);
      }
      const float b0 = bl[lo], b1 = bl[32 + lo];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = 32 * ti + 8 * (v >> 2) + 4 * hi + (v & 3);
        out(row, lo, acc0[v] + b0);
        out(row, 32 + lo, acc1[v] + b1);
      }
    }
  }
}

__device__ inline float standardised(double raw, float mean, float scale) {
  return (float)((raw - (double)mean) / (double)scale);
}

// x0 = u_prev + (mu_t + sigma_t y), rounded step by step
__device__ inline double start_value(double u, float mu, float sigma, float y) {
#pragma clang fp contract(off)
  return u + ((double)mu + (double)sigma * (double)y);
}

template <int NW>
__global__ __launch_bounds__(64 * NW, 1) void mlp_infer_kernel(int64_t P, const bf16* __restrict__ X,
                                                              const bf16* __restrict__ W,
                                                              const float* __restrict__ p32,
                                                              float* __restrict__ Y) {
  __shared__ __attribute__((aligned(16))) bf16 sH[kFR * kFLD];
  const int tid = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * kFR;
  {  // the input tile: 448 features = 56 chunks of 16 bytes per patch
    constexpr int CPR = WS_IN / 8;
    for (int c = tid; c < kFR * CPR; c += 64 * NW) {
      const int r = c / CPR, kc = (c % CPR) * 8;
      Vec16 v = Vec16{0u, 0u, 0u, 0u};
      if (p0 + r < P) v = *reinterpret_cast<const Vec16*>(X + (p0 + r) * WS_IN + kc);
      *reinterpret_cast<Vec16*>(&sH[r * kFLD + kc]) = v;
    }
  }
  __syncthreads();
  network_tile<NW>(sH, W, p32, [&](int row, int col, float y) {
    if (p0 + row < P) Y[(p0 + row) * WS_OUT + col] = y;
  });
}

// out[C, R] = in[R, C]^T through a 32 x 32 LDS tile.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(int64_t R, int64_t C,
                                                        const T* __restrict__ in,
                                                        T* __restrict__ out) {
  __shared__ T tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8)
    if (r0 + k < R && c0 + tx < C) tile[k][tx] = in[(r0 + k) * C + c0 + tx];
  __syncthreads();
  for (int k = ty; k < 32; k += 8)
    if (c0 + k < C && r0 + tx < R) out[(c0 + k) * R + r0 + tx] = tile[tx][k];
}

// Column sums in a fixed order: partial[g][n] over rows [256 g, 256 g + 256),
// then out[n] = sum_g partial[g][n].
template <typename T>
__global__ __launch_bounds__(256) void colsum_partial_kernel(int64_t M, int64_t N,
                                                             const T* __restrict__ in,
                                                             float* __restrict__ partial) {
  const int64_t n = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int q = threadIdx.x >> 6;  // 4 row groups of 64
  __shared__ float s[4][64];
  float acc = 0.0f;
  if (n < N) {
    const int64_t rb = (int64_t)blockIdx.y * 256 + q * 64;
    for (int k = 0; k < 64; ++k) {
      const int64_t m = rb + k;
      if (m < M) acc += (float)in[m * N + n];
    }
  }
  s[q][threadIdx.x & 63] = acc;
  __syncthreads();
  if (q == 0 && n < N)
    partial[(int64_t)blockIdx.y * N + n] = ((s[0][threadIdx.x] + s[1][threadIdx.x]) +
                                            s[2][threadIdx.x]) + s[3][threadIdx.x];
}

__global__ __launch_bounds__(256) void colsum_final_kernel(int64_t G, int64_t N,
                                                           const float* __restrict__ partial,
                                                           float* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  float acc = 0.0f;
  for (int64_t g = 0; g < G; ++g) acc += partial[g * N + n];
  out[n] = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void convert_kernel(int64_t count, const float* __restrict__ in,
                                                      T* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256)
    out[i] = (T)in[i];
}

__global__ __launch_bounds__(256) void mse_kernel(int64_t count, const float* __restrict__ Y,
                                                  const float* __restrict__ T,
                                                  float* __restrict__ dY,
                                                  double* __restrict__ partial) {
  __shared__ double s[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double sq = 0.0;
  if (i < count) {
    const float d = Y[i] - T[i];
    dY[i] = (float)(2.0 * (double)d / (double)count);
    sq = (double)d * (double)d;
  }
  s[threadIdx.x] = sq;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ void mse_final_kernel(int64_t G, int64_t count, const double* __restrict__ partial,
                                 double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc = 0.0;
  for (int64_t g = 0; g < G; ++g) acc += partial[g];
  *loss = acc / (double)count;
}

template <typename T>
__global__ __launch_bounds__(256) void adam_kernel(int64_t count, float* __restrict__ p,
                                                   T* __restrict__ pT,
                                                   const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (pT) pT[i] = (T)pi;
  }
}

struct Norm {
  float mean[7], scale[7];
};

// r0_i = rhs_i - (((d_i u_i + e_i u_{i-2}) + c_i u_{i-1}) + a_i u_{i+1}) + b_i u_{i+2}
// (terms outside the matrix omitted), every product and sum rounded on its
// own: the residual of the previous-step solution, the input through which the
// right-hand side reaches the network.
__device__ inline double residual_of(int64_t n, int64_t i, double e, double c, double d,
                                     double a, double b, double rhs, double um2, double um1,
                                     double u0, double up1, double up2) {
#pragma clang fp contract(off)
  double ax = d * u0;
  if (i >= 2) ax = ax + e * um2;
  if (i >= 1) ax = ax + c * um1;
  if (i <= n - 2) ax = ax + a * up1;
  if (i <= n - 3) ax = ax + b * up2;
  return rhs - ax;
}

__device__ inline double residual(int64_t n, int64_t ld, int64_t i, int64_t o,
                                  const double* __restrict__ E, const double* __restrict__ C,
                                  const double* __restrict__ D, const double* __restrict__ A,
                                  const double* __restrict__ B, double rhs,
                                  const double* __restrict__ U) {
  return residual_of(n, i, i >= 2 ? E[o] : 0.0, i >= 1 ? C[o] : 0.0, D[o],
                     i <= n - 2 ? A[o] : 0.0, i <= n - 3 ? B[o] : 0.0, rhs,
                     i >= 2 ? U[o - 2 * ld] : 0.0, i >= 1 ? U[o - ld] : 0.0, U[o],
                     i <= n - 2 ? U[o + ld] : 0.0, i <= n - 3 ? U[o + 2 * ld] : 0.0);
}

// One block: 64 systems x one patch row (64 rows); every feature plane goes
// through an LDS tile so that reads (consecutive systems) and writes
// (consecutive rows of a patch) are both contiguous.
template <typename T>
__global__ __launch_bounds__(256) void features_kernel(int64_t n, int64_t batch, int64_t ld,
                                                       const double* __restrict__ P0,
                                                       const double* __restrict__ P1,
                                                       const double* __restrict__ P2,
                                                       const double* __restrict__ P3,
                                                       const double* __restrict__ P4,
                                                       const double* __restrict__ P5,
                                                       const double* __restrict__ P6, Norm nm,
                                                       T* __restrict__ X) {
  __shared__ float tile[64][65];
  const int64_t s0 = (int64_t)blockIdx.x * 64, j = blockIdx.y;
  const int64_t npatch = (n + 63) / 64;
  const double* planes[7] = {P0, P1, P2, P3, P4, P5, P6};
  for (int f = 0; f < 7; ++f) {
    const double* P = planes[f];
    for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
      const int r = idx >> 6, sl = idx & 63;
      const int64_t i = j * 64 + r, s = s0 + sl;
      float val = 0.0f;
      if (i < n && s < batch) {
        const bool outside = (f == 0 && i < 2) || (f == 1 && i < 1) || (f == 3 && i > n - 2) ||
                             (f == 4 && i > n - 3);
        const int64_t o = i * ld + s;
        double raw = outside ? 0.0 : P[o];
        if (f == 5) raw = residual(n, ld, i, o, P0, P1, P2, P3, P4, raw, P6);
        val = standardised(raw, nm.mean[f], nm.scale[f]);
      }
      tile[r][sl] = val;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
      const int sl = idx >> 6, r = idx & 63;
      const int64_t s = s0 + sl;
      if (s < batch) X[(s * npatch + j) * 448 + f * 64 + r] = (T)tile[r][sl];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void apply_kernel(int64_t n, int64_t batch, int64_t ld,
                                                    const float* __restrict__ Y,
                                                    const double* __restrict__ U, float mu,
                                                    float sigma, double* __restrict__ X0) {
  __shared__ float tile[64][65];
  const int64_t s0 = (int64_t)blockIdx.x * 64, j = blockIdx.y;
  const int64_t npatch = (n + 63) / 64;
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int sl = idx >> 6, r = idx & 63;
    const int64_t s = s0 + sl;
    tile[r][sl] = s < batch ? Y[(s * npatch + j) * 64 + r] : 0.0f;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int r = idx >> 6, sl = idx & 63;
    const int64_t i = j * 64 + r, s = s0 + sl;
    if (i < n && s < batch) {
      const int64_t o = i * ld + s;
      X0[o] = start_value(U[o], mu, sigma, tile[r][sl]);
    }
  }
}

// features -> network -> start vector for one block of kFR consecutive
// systems and one patch row j (rows 64 j .. 64 j + 63), without X or Y going
// through memory.  The feature values are those of features_kernel (the same
// FP64 steps, rounded to FP32, then to bf16), written straight into the
// block's LDS tile; Y is staged in the LDS rows of its patches (each wave
// writes only rows it has finished reading) and x0 leaves row by row, so
// every load and store covers consecutive systems.  x0 equals ws_apply of the
// Y of ws_infer on the features of ws_features, bit for bit.
template <int NW>
__global__ __launch_bounds__(64 * NW, 1) void predict_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ P0,
    const double* __restrict__ P1, const double* __restrict__ P2, const double* __restrict__ P3,
    const double* __restrict__ P4, const double* __restrict__ P5, const double* __restrict__ P6,
    Norm nm, const bf16* __restrict__ W, const float* __restrict__ p32, float mu, float sigma,
    double* __restrict__ X0) {
  __shared__ __attribute__((aligned(16))) bf16 sH[kFR * kFLD];
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * kFR, j = blockIdx.y;
  // UB elements per thread at a time, all their loads issued before the
  // arithmetic (11 loads each: the seven planes and u_prev at i -+ 1, 2)
  constexpr int EPT = 64 * kFR / (64 * NW), UB = 4;
  static_assert(EPT % UB == 0, "elements per thread");
  const double* planes[7] = {P0, P1, P2, P3, P4, P5, P6};
  for (int e0 = 0; e0 < EPT; e0 += UB) {
    double v[UB][7], um2[UB], um1[UB], up1[UB], up2[UB];
    int64_t ii[UB];
    bool in[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int idx = tid + (e0 + u) * 64 * NW;
      const int r = idx / kFR, sl = idx % kFR;  // consecutive threads: consecutive systems
      const int64_t i = j * 64 + r, s = s0 + sl, o = i * ld + s;
      ii[u] = i;
      in[u] = i < n && s < batch;
#pragma unroll
      for (int f = 0; f < 7; ++f) {
        const bool outside = (f == 0 && i < 2) || (f == 1 && i < 1) || (f == 3 && i > n - 2) ||
                             (f == 4 && i > n - 3);
        v[u][f] = (in[u] && !outside) ? __builtin_nontemporal_load(planes[f] + o) : 0.0;
      }
      um2[u] = (in[u] && i >= 2) ? P6[o - 2 * ld] : 0.0;
      um1[u] = (in[u] && i >= 1) ? P6[o - ld] : 0.0;
      up1[u] = (in[u] && i <= n - 2) ? P6[o + ld] : 0.0;
      up2[u] = (in[u] && i <= n - 3) ? P6[o + 2 * ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int idx = tid + (e0 + u) * 64 * NW;
      const int r = idx / kFR, sl = idx % kFR;
#pragma unroll
      for (int f = 0; f < 7; ++f) {
        float val = 0.0f;
        if (in[u]) {
          const double raw = f == 5 ? residual_of(n, ii[u], v[u][0], v[u][1], v[u][2], v[u][3],
                                                  v[u][4], v[u][5], um2[u], um1[u], v[u][6],
                                                  up1[u], up2[u])
                                    : v[u][f];
          val = standardised(raw, nm.mean[f], nm.scale[f]);
        }
        // the FP32 value first, then bf16 (as features_kernel, which stores
        // the FP32 value in between): without the barrier the compiler folds
        // the two conversions into one correctly rounded FP64 -> bf16
        // conversion, which differs from the double rounding where the FP32
        // value is a bf16 tie
        asm volatile("" : "+v"(val));
        sH[sl * kFLD + f * 64 + r] = (bf16)val;
      }
    }
  }
  __syncthreads();
  float* yS = reinterpret_cast<float*>(sH);  // patch row sl at yS[sl * kFLD / 2 + r]
  network_tile<NW>(sH, W, p32, [&](int row, int col, float y) { yS[row * (kFLD / 2) + col] = y; });
  __syncthreads();
  for (int idx = tid; idx < 64 * kFR; idx += 64 * NW) {
    const int r = idx / kFR, sl = idx % kFR;
    const int64_t i = j * 64 + r, s = s0 + sl;
    if (i < n && s < batch) {
      const int64_t o = i * ld + s;
      X0[o] = start_value(P6[o], mu, sigma, yS[sl * (kFLD / 2) + r]);
    }
  }
}

// ---------------------------------------------------------------- host ---
int grid1(int64_t work) {
  const int64_t b = (work + 255) / 256;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

bool al16(const void* p) { return p != nullptr && (reinterpret_cast<uintptr_t>(p) & 15) == 0; }
size_t esz(int32_t dtype) { return dtype == WS_BF16 ? 2 : 4; }
bool dtype_ok(int32_t dtype) { return dtype == WS_BF16 || dtype == WS_F32; }

template <typename T, int TI, int TJ>
hipError_t gemm_tiles(int64_t M, int64_t N, int64_t K, const void* A, const void* B,
                      const float* bias, int relu, const void* mask, float* C32, void* CT,
                      hipStream_t st) {
  constexpr int BM = 64 * TI, BN = 64 * TJ;
  const dim3 grid((unsigned)(((N + BN - 1) / BN) * ((M + BM - 1) / BM)));
  hipLaunchKernelGGL((gemm_nt_kernel<T, TI, TJ>), grid, dim3(kThreads), 0, st, M, N, K,
                     static_cast<const T*>(A), static_cast<const T*>(B), bias, relu,
                     static_cast<const T*>(mask), C32, static_cast<T*>(CT));
  return hipGetLastError();
}

// 128 x 128 blocks (2 x 2 MFMA tiles per wave).  Measured on the 262144 x 512
// x 512 layer: 256 x 128 blocks (4 x 2 per wave, one block per CU) ran 1.3x
// slower than these, which keep two blocks per CU.
template <typename T>
hipError_t gemm(int64_t M, int64_t N, int64_t K, const void* A, const void* B, const float* bias,
                int relu, const void* mask, float* C32, void* CT, hipStream_t st) {
  return gemm_tiles<T, 2, 2>(M, N, K, A, B, bias, relu, mask, C32, CT, st);
}

template <typename T>
void transpose(int64_t R, int64_t C, const void* in, void* out, hipStream_t st) {
  const dim3 grid((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32));
  hipLaunchKernelGGL(transpose_kernel<T>, grid, dim3(256), 0, st, R, C,
                     static_cast<const T*>(in), static_cast<T*>(out));
}

template <typename T>
void colsum(int64_t M, int64_t N, const void* in, float* partial, float* out, hipStream_t st) {
  const int64_t G = (M + 255) / 256;
  hipLaunchKernelGGL(colsum_partial_kernel<T>, dim3((unsigned)((N + 63) / 64), (unsigned)G),
                     dim3(256), 0, st, M, N, static_cast<const T*>(in), partial);
  hipLaunchKernelGGL(colsum_final_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                     G, N, partial, out);
}

// Parameter offsets (elements) of layer k: W then b.
struct Layer {
  int64_t in, out, w, b;
};
constexpr int kLayers = 4;
void layers(Layer L[kLayers]) {
  const int64_t dims[5] = {WS_IN, WS_HIDDEN, WS_HIDDEN, WS_HIDDEN, WS_OUT};
  int64_t o = 0;
  for (int k = 0; k < kLayers; ++k) {
    L[k].in = dims[k];
    L[k].out = dims[k + 1];
    L[k].w = o;
    o += L[k].in * L[k].out;
    L[k].b = o;
    o += L[k].out;
  }
}
int64_t param_count() {
  Layer L[kLayers];
  layers(L);
  return L[kLayers - 1].b + L[kLayers - 1].out;
}

// Workspace: h1, h2, h3 [P, WS_HIDDEN] (forward); then for training dY in
// dtype [P, 64], two [WS_HIDDEN, P] transposes, two [P, WS_HIDDEN] gradient
// buffers, a [WS_HIDDEN, WS_HIDDEN] weight transpose and the column-sum
// partials.
struct WsLayout {
  size_t h[3], dyT, ta, tb, ga, gb, wt, part, fwd_total, train_total;
};
WsLayout ws_layout(int32_t dtype, int64_t P) {
  WsLayout L;
  const size_t e = esz(dtype);
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  size_t o = 0;
  for (int k = 0; k < 3; ++k) {
    L.h[k] = o;
    o = up(o + (size_t)P * WS_HIDDEN * e);
  }
  L.fwd_total = o;
  L.dyT = o;  o = up(o + (size_t)P * WS_OUT * e);
  L.ta = o;   o = up(o + (size_t)P * WS_HIDDEN * e);
  L.tb = o;   o = up(o + (size_t)P * WS_HIDDEN * e);
  L.ga = o;   o = up(o + (size_t)P * WS_HIDDEN * e);
  L.gb = o;   o = up(o + (size_t)P * WS_HIDDEN * e);
  L.wt = o;   o = up(o + (size_t)WS_HIDDEN * WS_HIDDEN * e);
  L.part = o; o = up(o + (size_t)((P + 255) / 256) * WS_HIDDEN * 4);
  L.train_total = o;
  return L;
}

template <typename T>
hipError_t forward(int64_t P, const void* X, const float* p32, const void* pT, float* Y,
                   char* ws, hipStream_t st) {
  Layer L[kLayers];
  layers(L);
  const WsLayout W = ws_layout(sizeof(T) == 2 ? WS_BF16 : WS_F32, P);
  const T* w = static_cast<const T*>(pT);
  const void* in = X;
  for (int k = 0; k < kLayers; ++k) {
    const bool last = k == kLayers - 1;
    void* out = last ? nullptr : ws + W.h[k];
    hipError_t e = gemm<T>(P, L[k].out, L[k].in, in, w + L[k].w, p32 + L[k].b, last ? 0 : 1,
                           nullptr, last ? Y : nullptr, out, st);
    if (e != hipSuccess) return e;
    in = out;
  }
  return hipSuccess;
}

template <typename T>
hipError_t backward(int64_t P, const void* X, const void* pT, const float* dY, float* g,
                    char* ws, hipStream_t st) {
  Layer L[kLayers];
  layers(L);
  const WsLayout W = ws_layout(sizeof(T) == 2 ? WS_BF16 : WS_F32, P);
  const T* w = static_cast<const T*>(pT);
  float* part = reinterpret_cast<float*>(ws + W.part);
  // output layer: gradient operand in dtype, bias gradient from FP32 dY
  T* gcur = reinterpret_cast<T*>(ws + W.dyT);
  hipLaunchKernelGGL(convert_kernel<T>, dim3(grid1(P * WS_OUT)), dim3(256), 0, st, P * WS_OUT,
                     dY, gcur);
  colsum<float>(P, WS_OUT, dY, part, g + L[3].b, st);
  T* gbuf[2] = {reinterpret_cast<T*>(ws + W.ga), reinterpret_cast<T*>(ws + W.gb)};
  for (int k = kLayers - 1; k >= 0; --k) {
    const int64_t out = L[k].out, in = L[k].in;
    const void* hin = k == 0 ? X : ws + W.h[k - 1];
    if (k < kLayers - 1) colsum<T>(P, out, gcur, part, g + L[k].b, st);
    // dW_k [out, in] = g^T [out, P] (h_in^T [in, P])^T
    transpose<T>(P, out, gcur, ws + W.ta, st);
    transpose<T>(P, in, hin, ws + W.tb, st);
    hipError_t e = gemm<T>(out, in, P, ws + W.ta, ws + W.tb, nullptr, 0, nullptr, g + L[k].w,
                           nullptr, st);
    if (e != hipSuccess) return e;
    if (k == 0) break;
    // g_{k-1} [P, in] = (g [P, out] W_k [out, in]) * [h_{k-1} > 0];  W_k^T is [in, out]
    transpose<T>(out, in, w + L[k].w, ws + W.wt, st);
    T* gnext = gbuf[k & 1];
    e = gemm<T>(P, in, out, gcur, ws + W.wt, nullptr, 0, ws + W.h[k - 1], nullptr, gnext, st);
    if (e != hipSuccess) return e;
    gcur = gnext;
  }
  return hipGetLastError();
}

}  // namespace
}  // namespace wsm

using namespace wsm;

extern "C" {

int64_t ws_param_count(void) { return param_count(); }

size_t ws_workspace_bytes(int32_t op, int32_t dtype, int64_t P) {
  if (!dtype_ok(dtype) || P < 1 || P > (int64_t(1) << 31)) return (size_t)-1;
  const WsLayout L = ws_layout(dtype, P);
  if (op == WS_OP_FORWARD) return L.fwd_total;
  if (op == WS_OP_TRAIN) return L.train_total;
  return (size_t)-1;
}

int32_t ws_gemm_nt(int32_t dtype, int64_t M, int64_t N, int64_t K, const void* A, const void* B,
                   const float* bias, int32_t relu, const void* mask, float* C32, void* CT,
                   void* stream) {
  if (!dtype_ok(dtype) || M < 1 || N < 1 || K < 1) return BS_EINVAL;
  if (K % (int64_t)(16 / esz(dtype)) != 0) return BS_EINVAL;
  if (M > (int64_t(1) << 31) || N > (int64_t(1) << 31) || (M + 127) / 128 > 65535)
    return BS_EINVAL;
  if (!al16(A) || !al16(B) || (C32 == nullptr && CT == nullptr)) return BS_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = dtype == WS_BF16 ? gemm<bf16>(M, N, K, A, B, bias, relu, mask, C32, CT, st)
                                  : gemm<float>(M, N, K, A, B, bias, relu, mask, C32, CT, st);
  return e == hipSuccess ? BS_OK : BS_ELAUNCH;
}

int32_t ws_convert(int32_t dtype, int64_t count, const float* in, void* out, void* stream) {
  if (!dtype_ok(dtype) || count < 0 || !al16(in) || !al16(out)) return BS_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == WS_BF16)
    hipLaunchKernelGGL(convert_kernel<bf16>, dim3(grid1(count)), dim3(256), 0, st, count, in,
                       static_cast<bf16*>(out));
  else
    hipLaunchKernelGGL(convert_kernel<float>, dim3(grid1(count)), dim3(256), 0, st, count, in,
                       static_cast<float*>(out));
  return hipGetLastError() == hipSuccess ? BS_OK : BS_ELAUNCH;
}

int32_t ws_forward(int32_t dtype, int64_t P, const void* X, const float* params32,
                   const void* paramsT, float* Y, void* workspace, size_t ws_bytes,
                   void* stream) {
  const size_t need = ws_workspace_bytes(WS_OP_FORWARD, dtype, P);
  if (need == (size_t)-1 || (P + 127) / 128 > 65535) return BS_EINVAL;
  if (!al16(X) || !al16(params32) || !al16(paramsT) || !al16(Y) || !al16(workspace))
    return BS_EINVAL;
  if (ws_bytes < need) return BS_EWORKSPACE;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  hipError_t e = dtype == WS_BF16 ? forward<bf16>(P, X, params32, paramsT, Y, ws, st)
                                  : forward<float>(P, X, params32, paramsT, Y, ws, st);
  return e == hipSuccess ? BS_OK : BS_ELAUNCH;
}

int32_t ws_infer(int64_t P, const void* X, const float* params32, const void* paramsT, float* Y,
                 void* stream) {
  if (P < 1 || P > (int64_t(1) << 31) || (P + kFR - 1) / kFR > (int64_t(1) << 31) - 1)
    return BS_EINVAL;
  if (!al16(X) || !al16(params32) || !al16(paramsT) || !al16(Y)) return BS_EINVAL;
  hipLaunchKernelGGL(mlp_infer_kernel<kInferWaves>, dim3((unsigned)((P + kFR - 1) / kFR)),
                     dim3(64 * kInferWaves), 0, static_cast<hipStream_t>(stream), P,
                     static_cast<const bf16*>(X), static_cast<const bf16*>(paramsT), params32, Y);
  return hipGetLastError() == hipSuccess ? BS_OK : BS_ELAUNCH;
}

int32_t ws_backward(int32_t dtype, int64_t P, const void* X, const float* params32,
                    const void* paramsT, const float* dY, float* grads, void* workspace,
                    size_t ws_bytes, void* stream) {
  const size_t need = ws_workspace_bytes(WS_OP_TRAIN, dtype, P);
  if (need == (size_t)-1 || P % 8 != 0 || (P + 127) / 128 > 65535) return BS_EINVAL;
  if (!al16(X) || !al16(params32) || !al16(paramsT) || !al16(dY) || !al16(grads) ||
      !al16(workspace))
    return BS_EINVAL;
  if (ws_bytes < need) return BS_EWORKSPACE;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  hipError_t e = dtype == WS_BF16 ? backward<bf16>(P, X, paramsT, dY, grads, ws, st)
                                  : backward<float>(P, X, paramsT, dY, grads, ws, st);
  return e == hipSuccess ? BS_OK : BS_ELAUNCH;
}

int32_t ws_mse(int64_t P, const float* Y, const float* T, float* dY, double* loss,
               double* partial, void* stream) {
  if (P < 1 || !al16(Y) || !al16(T) || !al16(dY) || loss == nullptr || partial == nullptr)
    return BS_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t count = P * WS_OUT;
  const int64_t G = (count + 255) / 256;
  hipLaunchKernelGGL(mse_kernel, dim3((unsigned)G), dim3(256), 0, st, count, Y, T, dY, partial);
  hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(64), 0, st, G, count, partial, loss);
  return hipGetLastError() == hipSuccess ? BS_OK : BS_ELAUNCH;
}

int32_t ws_adam(int32_t dtype, int64_t count, float* params, void* paramsT, const float* grads,
                float* m, float* v, float lr, float beta1, float beta2, float eps, int32_t step,
                void* stream) {
  if (!dtype_ok(dtype) || count < 1 || step < 1 || !al16(params) || !al16(grads) || !al16(m) ||
      !al16(v))
    return BS_EINVAL;
  if (paramsT != nullptr && !al16(paramsT)) return BS_EINVAL;
  const float c1 = (float)(1.0 - std::pow((double)beta1, step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, step));
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == WS_BF16)
    hipLaunchKernelGGL(adam_kernel<bf16>, dim3(grid1(count)), dim3(256), 0, st, count, params,
                       static_cast<bf16*>(paramsT), grads, m, v, lr, beta1, beta2, eps, c1, c2);
  else
    hipLaunchKernelGGL(adam_kernel<float>, dim3(grid1(count)), dim3(256), 0, st, count, params,
                       static_cast<float*>(paramsT), grads, m, v, lr, beta1, beta2, eps, c1,
                       c2);
  return hipGetLastError() == hipSuccess ? BS_OK : BS_ELAUNCH;
}

int32_t ws_features(int32_t dtype, int64_t n, int64_t batch, int64_t ld,
                    const double* const planes[7], const float norm[14], void* X,
                    void* stream) {
  if (!dtype_ok(dtype) || n < 1 || batch < 1 || ld < batch || planes == nullptr ||
      norm == nullptr || !al16(X))
    return BS_EINVAL;
  if ((n + 63) / 64 > 65535) return BS_EINVAL;
  Norm nm;
  for (int f = 0; f < 7; ++f) {
    if (planes[f] == nullptr || !(norm[7 + f] > 0.0f)) return BS_EINVAL;
    nm.mean[f] = norm[f];
    nm.scale[f] = norm[7 + f];
  }
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid((unsigned)((batch + 63) / 64), (unsigned)((n + 63) / 64));
  if (dtype == WS_BF16)
    hipLaunchKernelGGL(features_kernel<bf16>, grid, dim3(256), 0, st, n, batch, ld, planes[0],
                       planes[1], planes[2], planes[3], planes[4], planes[5], planes[6], nm,
                       static_cast<bf16*>(X));
  else
    hipLaunchKernelGGL(features_kernel<float>, grid, dim3(256), 0, st, n, batch, ld, planes[0],
                       planes[1], planes[2], planes[3], planes[4], planes[5], planes[6], nm,
                       static_cast<float*>(X));
  return hipGetLastError() == hipSuccess ? BS_OK : BS_ELAUNCH;
}

int32_t ws_apply(int64_t n, int64_t batch, int64_t ld, const float* Y, const double* uprev,
                 float mu_t, float sigma_t, double* x0, void* stream) {
  if (n < 1 || batch < 1 || ld < batch || !al16(Y) || uprev == nullptr || x0 == nullptr)
    return BS_EINVAL;
  if ((n + 63) / 64 > 65535) return BS_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid((unsigned)((batch + 63) / 64), (unsigned)((n + 63) / 64));
  hipLaunchKernelGGL(apply_kernel, grid, dim3(256), 0, st, n, batch, ld, Y, uprev, mu_t, sigma_t,
                     x0);
  return hipGetLastError() == hipSuccess ? BS_OK : BS_ELAUNCH;
}

int32_t ws_predict(int64_t n, int64_t batch, int64_t ld, const double* const planes[7],
                   const float norm[14], const float* params32, const void* paramsT, float mu_t,
                   float sigma_t, double* x0, void* stream) {
  if (n < 1 || batch < 1 || ld < batch || planes == nullptr || norm == nullptr ||
      !al16(params32) || !al16(paramsT) || x0 == nullptr)
    return BS_EINVAL;
  if ((n + 63) / 64 > 65535 || (batch + kFR - 1) / kFR > (int64_t(1) << 31) - 1) return BS_EINVAL;
  Norm nm;
  for (int f = 0; f < 7; ++f) {
    if (planes[f] == nullptr || !(norm[7 + f] > 0.0f)) return BS_EINVAL;
    nm.mean[f] = norm[f];
    nm.scale[f] = norm[7 + f];
  }
  const dim3 grid((unsigned)((batch + kFR - 1) / kFR), (unsigned)((n + 63) / 64));
  hipLaunchKernelGGL(predict_kernel<kInferWaves>, grid, dim3(64 * kInferWaves), 0,
                     static_cast<hipStream_t>(stream), n, batch, ld, planes[0], planes[1],
                     planes[2], planes[3], planes[4], planes[5], planes[6], nm,
                     static_cast<const bf16*>(paramsT), params32, mu_t, sigma_t, x0);
  return hipGetLastError() == hipSuccess ? BS_OK : BS_ELAUNCH;
}

}  // extern "C"
