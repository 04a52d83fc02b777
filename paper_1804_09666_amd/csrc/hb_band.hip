// hb_band.hip -- the Hotelling-Bodewig approximate inverses of the ILU(0)
// factors as explicit band matrices (Veneva & Ayriyan, arXiv:1804.09666:
// the Remark of Sec. 2 and the HB equation of the Appendix, whose tables time
// L^{-1} and U^{-1} in the matrix form):
//   X_0 = diag(T)^{-1},   X_{j+1} = X_j (2 I - T X_j),   j < s,
// for T = L (unit lower, l2 and l1 below the diagonal) and T = U (u0 on the
// diagonal, u1 and u2 = b above it; for a tridiagonal band l1 and u0, u1 = a).
// X_j is a band matrix of width q (2^j - 1), q the factor's bandwidth (2 for
// a pentadiagonal band, 1 for a tridiagonal one): T has width q, so T X_j has
// width b_j + q and X_j M width 2 b_j + q = b_{j+1}.
//
// Every product is summed over its inner index in ascending order, one
// rounded multiply and one rounded add per term (no contraction), from an
// accumulator of zero: terms outside the bands are exact zeros and change no
// sum, so the band entries are those of the same recursion on dense
// matrices.  A step whose output band is narrower than 16 is one launch that
// forms M = 2 I - T X_j in registers inside the product; a wider one is two
// launches, M into the workspace, then X_{j+1} = X_j M.  Entries are stored
// by distance from the diagonal:
// plane d of a lower factor holds X[i, i - d] at d*n*ld + i*ld + s, plane d
// of an upper one X[i, i + d]; slots outside the matrix hold 0.
#include <type_traits>

#include "bandsolve.h"
#include "bs_internal.h"

namespace bs {
namespace {

constexpr int kBlock = 256;
#ifndef HB_XT_R
#define HB_XT_R 4  // rows per lane in the product step
#endif
#ifndef HB_XT_D
#define HB_XT_D 16  // distances per lane in the product step (wide bands)
#endif

struct Tri {  // the factor T: diagonal (null: unit), then q off-diagonals
  const double* dg;
  const double* o1;  // first off-diagonal (l1 below / u1 above)
  const double* o2;  // second off-diagonal (l2 / u2), null when q = 1
};

// Work-item layout shared by the step kernels: a block is four waves; lane =
// system within a group of 64, wave = row tile within the block's four.  The
// row, distance and plane arithmetic is wave-uniform (scalar registers), so
// a lane's only private address part is its byte offset 8 s.
struct Item {
  int64_t chunk, tile, s;
  uint32_t boff;  // byte offset of the lane's system (clamped to a live one)
  bool live;
};

__device__ inline Item work_item(int64_t batch, int64_t tiles, int64_t chunks, int64_t work) {
  int64_t w = blockIdx.x;
  if (work % 8 == 0) w = (w % 8) * (work / 8) + w / 8;  // XCD-contiguous work ranges
  Item it;
  it.chunk = w % chunks;
  const int64_t rest = w / chunks;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  it.tile = (rest % tiles) * 4 + wave;
  it.s = (rest / tiles) * 64 + (threadIdx.x & 63);
  it.live = it.s < batch;
  it.boff = (uint32_t)((it.live ? it.s : batch - 1) * 8);
  return it;
}

__device__ inline double at(const double* base, int64_t uniform_off, uint32_t boff) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base + uniform_off) +
                                          boff);
}
__device__ inline void put(double* base, int64_t uniform_off, uint32_t boff, double v) {
  *reinterpret_cast<double*>(reinterpret_cast<char*>(base + uniform_off) + boff) = v;
}

// X_0 = diag(T)^{-1} into plane 0.
__global__ __launch_bounds__(kBlock) void hb_init_kernel(int64_t n, int64_t batch, int64_t ld,
                                                         Tri T, double* __restrict__ X) {
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n * batch;
       q += (int64_t)gridDim.x * kBlock) {
    const int64_t s = q % batch, i = q / batch, o = i * ld + s;
    X[o] = 1.0 / (T.dg ? T.dg[o] : 1.0);
  }
}

// M = 2 I - T X_j (band bm = bx + q).  A lane forms D consecutive distances
// of one row: (T X_j)[i, k] takes its q + 1 terms in ascending inner index l
// (X_j entries outside its band enter as zeros), then M = 2 delta - (T X_j).
template <bool LOWER, int D>
__global__ __launch_bounds__(kBlock) void hb_m_kernel(int64_t n, int64_t batch, int64_t ld,
                                                      Tri T, int q, const double* __restrict__ X,
                                                      int64_t bx, double* __restrict__ Mb,
                                                      int64_t bm, int64_t tiles, int64_t chunks,
                                                      int64_t work) {
#pragma clang fp contract(off)
  const Item it = work_item(batch, tiles, chunks, work);
  const int64_t i = it.tile, d0 = it.chunk * D, plane = n * ld;
  if (i >= n) return;
  // t[m]: T[i, l] for the m-th inner index l in ascending order
  double t[3];
  const int64_t lbeg = LOWER ? i - q : i;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const int64_t l = lbeg + m;
    const int64_t dist = LOWER ? i - l : l - i;
    t[m] = 0.0;
    if (m <= q && l >= 0 && l < n) {
      const double* src = dist == 0 ? T.dg : (dist == 1 ? T.o1 : T.o2);
      t[m] = src ? at(src, i * ld, it.boff) : 1.0;
    }
  }
  double acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const int64_t l = lbeg + m;
    if (m > q || l < 0 || l >= n) continue;
    // X_j[l, k] for k = i -+ d lies at distance e = d - (i - l) (lower) or
    // d - (l - i) (upper) from row l's diagonal
    const int64_t shift = LOWER ? i - l : l - i;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const int64_t e = d0 + c - shift;
      const double x = (e >= 0 && e <= bx) ? at(X, e * plane + l * ld, it.boff) : 0.0;
      acc[c] = acc[c] + t[m] * x;
    }
  }
  if (!it.live) return;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const int64_t d = d0 + c;
    if (d > bm) break;
    const int64_t k = LOWER ? i - d : i + d;
    const double v = (k >= 0 && k < n) ? (d == 0 ? 2.0 : 0.0) - acc[c] : 0.0;
    put(Mb, d * plane + i * ld, it.boff, v);
  }
}

// X_{j+1} = X_j M, register-tiled: a lane owns one system, R consecutive
// rows and D consecutive distances d0 .. d0 + D - 1.  It sweeps the inner
// index l upwards once; at each l it loads the R entries X[i, l] of its rows
// and the D + R - 1 entries of M's row l that those rows need, then updates
// the R x D sums.  Entries outside a band or the matrix enter as zeros, which
// leave a sum unchanged (a sum that starts at +0 is never -0), so each output
// still takes its terms in ascending l with one rounding per multiply and add.
template <bool LOWER, int R, int D>
__global__ __launch_bounds__(kBlock) void hb_xt_kernel(int64_t n, int64_t batch, int64_t ld,
                                                       const double* __restrict__ X, int64_t bx,
                                                       const double* __restrict__ Mb, int64_t bm,
                                                       double* __restrict__ Xo, int64_t bo,
                                                       int64_t tiles, int64_t chunks,
                                                       int64_t work) {
#pragma clang fp contract(off)
  const Item it = work_item(batch, tiles, chunks, work);
  const int64_t i0 = it.tile * R, d0 = it.chunk * D, plane = n * ld;
  if (i0 >= n) return;
  const int64_t elo = d0 - bm > 0 ? d0 - bm : 0;
  const int64_t ehi = bx < d0 + D - 1 ? bx : d0 + D - 1;
  int64_t lfirst = LOWER ? i0 - ehi : i0 + elo;
  int64_t llast = LOWER ? i0 + R - 1 - elo : i0 + R - 1 + ehi;
  if (lfirst < 0) lfirst = 0;
  if (llast > n - 1) llast = n - 1;
  double acc[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int t = 0; t < D; ++t) acc[r][t] = 0.0;
  for (int64_t l = lfirst; l <= llast; ++l) {
    double xr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = i0 + r;
      const int64_t e = LOWER ? i - l : l - i;
      xr[r] = (e >= 0 && e <= bx && i < n) ? at(X, e * plane + i * ld, it.boff) : 0.0;
    }
    // window entry v holds M at distance f = fb + v from row l
    const int64_t fb = LOWER ? d0 - i0 + l - (R - 1) : d0 - (l - i0);
    double mw[D + R - 1];
#pragma unroll
    for (int v = 0; v < D + R - 1; ++v) {
      const int64_t f = fb + v;
      mw[v] = (f >= 0 && f <= bm) ? at(Mb, f * plane + l * ld, it.boff) : 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int t = 0; t < D; ++t) {
        const double m = LOWER ? mw[t - r + R - 1] : mw[t + r];
        acc[r][t] = acc[r][t] + xr[r] * m;
      }
  }
  if (!it.live) return;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = i0 + r;
    if (i >= n) break;
#pragma unroll
    for (int t = 0; t < D; ++t) {
      const int64_t d = d0 + t;
      if (d > bo) break;
      const int64_t k = LOWER ? i - d : i + d;
      put(Xo, d * plane + i * ld, it.boff, (k >= 0 && k < n) ? acc[r][t] : 0.0);
    }
  }
}

// X_{j+1} = X_j M with M = 2 I - T X_j formed in registers, never stored.
// In the sweep over l, the M entries a lane needs in row l sit at distances
// fb + v (v < W = D + R - 1), and M[l, k] takes X_j rows l .. l + q (upper;
// l - q .. l below the diagonal) at column k.  For a fixed row rho of X_j
// those columns are one window of W planes whatever l is, so each X_j row
// window is loaded once and kept for the q + 1 values of l that use it (a
// ring of q + 1 windows).  Every M entry is the M kernel's: (T X_j)[l, k]
// over the inner index in ascending order, then 2 delta - (T X_j), so the
// result is bitwise the two-kernel step.
template <bool LOWER, int Q, int R, int D>
__global__ __launch_bounds__(kBlock) void hb_xf_kernel(int64_t n, int64_t batch, int64_t ld,
                                                       Tri T, const double* __restrict__ X,
                                                       int64_t bx, int64_t bm,
                                                       double* __restrict__ Xo, int64_t bo,
                                                       int64_t tiles, int64_t chunks,
                                                       int64_t work) {
#pragma clang fp contract(off)
  constexpr int W = D + R - 1, NR = Q + 1;
  const Item it = work_item(batch, tiles, chunks, work);
  const int64_t i0 = it.tile * R, d0 = it.chunk * D, plane = n * ld;
  if (i0 >= n) return;
  const int64_t elo = d0 - bm > 0 ? d0 - bm : 0;
  const int64_t ehi = bx < d0 + D - 1 ? bx : d0 + D - 1;
  int64_t lfirst = LOWER ? i0 - ehi : i0 + elo;
  int64_t llast = LOWER ? i0 + R - 1 - elo : i0 + R - 1 + ehi;
  if (lfirst < 0) lfirst = 0;
  if (llast > n - 1) llast = n - 1;
  double acc[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int t = 0; t < D; ++t) acc[r][t] = 0.0;
  // window of X_j row rho: planes pb(rho) + v (0 outside the band or matrix)
  auto load_win = [&](int64_t rho, double (&xw)[W]) {
    const int64_t pb = LOWER ? rho + d0 - i0 - (R - 1) : d0 + i0 - rho;
#pragma unroll
    for (int v = 0; v < W; ++v) {
      const int64_t e = pb + v;
      xw[v] = (rho >= 0 && rho < n && e >= 0 && e <= bx) ? at(X, e * plane + rho * ld, it.boff)
                                                         : 0.0;
    }
  };
  double ring[NR][W];
  // the ring slot of the window of the m-th inner row at rotation K
  const int64_t rho0 = LOWER ? lfirst - Q : lfirst;  // inner row m = 0 at l = lfirst
  if (lfirst <= llast) {
#pragma unroll
    for (int m = 0; m < Q; ++m) load_win(rho0 + m, ring[m]);
  }
  auto body = [&](auto Kc, int64_t l) {
    constexpr int K = decltype(Kc)::value;
    load_win(LOWER ? l : l + Q, ring[(K + Q) % NR]);
    // T[l, inner row m], m ascending (0 where the inner row is outside)
    double t[NR];
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      const int64_t rho = LOWER ? l - Q + m : l + m;
      const int dist = LOWER ? Q - m : m;
      const double* src = dist == 0 ? T.dg : (dist == 1 ? T.o1 : T.o2);
      t[m] = (rho >= 0 && rho < n) ? (src ? at(src, l * ld, it.boff) : 1.0) : 0.0;
    }
    double xr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = i0 + r;
      const int64_t e = LOWER ? i - l : l - i;
      xr[r] = (e >= 0 && e <= bx && i < n) ? at(X, e * plane + i * ld, it.boff) : 0.0;
    }
    const int64_t fb = LOWER ? d0 - i0 + l - (R - 1) : d0 - (l - i0);
#pragma unroll
    for (int v = 0; v < W; ++v) {
      double tx = 0.0;
#pragma unroll
      for (int m = 0; m < NR; ++m) tx = tx + t[m] * ring[(K + m) % NR][v];
      const double mv = (fb + v == 0 ? 2.0 : 0.0) - tx;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int tt = LOWER ? v + r - (R - 1) : v - r;
        if (tt >= 0 && tt < D) acc[r][tt] = acc[r][tt] + xr[r] * mv;
      }
    }
  };
  int64_t l = lfirst;
  for (; l + Q <= llast; l += NR) {
    body(std::integral_constant<int, 0>{}, l);
    body(std::integral_constant<int, 1>{}, l + 1);
    if constexpr (Q == 2) body(std::integral_constant<int, 2>{}, l + 2);
  }
  if (l <= llast) body(std::integral_constant<int, 0>{}, l);
  if constexpr (Q == 2)
    if (l + 1 <= llast) body(std::integral_constant<int, 1>{}, l + 1);
  if (!it.live) return;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = i0 + r;
    if (i >= n) break;
#pragma unroll
    for (int t = 0; t < D; ++t) {
      const int64_t d = d0 + t;
      if (d > bo) break;
      const int64_t k = LOWER ? i - d : i + d;
      put(Xo, d * plane + i * ld, it.boff, (k >= 0 && k < n) ? acc[r][t] : 0.0);
    }
  }
}

int grid_for(int64_t work) {
  const int64_t b = (work + kBlock - 1) / kBlock;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

int64_t band_width(int q, int s, int64_t n) {
  if (s >= 62) return n - 1;
  const int64_t w = (int64_t)q * ((int64_t(1) << s) - 1);
  return w < n - 1 ? w : n - 1;
}

template <bool LOWER, int R, int D>
hipError_t launch_xt_rd(int64_t n, int64_t batch, int64_t ld, const double* X, int64_t bx,
                        const double* Mb, int64_t bm, double* Xo, int64_t bo, hipStream_t st) {
  const int64_t tiles = (n + 4 * R - 1) / (4 * R);
  const int64_t chunks = (bo + D) / D;
  const int64_t work = ((batch + 63) / 64) * tiles * chunks;
  if (work > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((hb_xt_kernel<LOWER, R, D>), dim3((unsigned)work), dim3(kBlock), 0, st, n,
                     batch, ld, X, bx, Mb, bm, Xo, bo, tiles, chunks, work);
  return hipGetLastError();
}

// Tile shape by the output band: D covers it where it is narrow.
template <bool LOWER>
hipError_t launch_xt(int64_t n, int64_t batch, int64_t ld, const double* X, int64_t bx,
                     const double* Mb, int64_t bm, double* Xo, int64_t bo, hipStream_t st) {
  if (bo < 4) return launch_xt_rd<LOWER, 4, 4>(n, batch, ld, X, bx, Mb, bm, Xo, bo, st);
  if (bo < 8) return launch_xt_rd<LOWER, 4, 8>(n, batch, ld, X, bx, Mb, bm, Xo, bo, st);
  return launch_xt_rd<LOWER, HB_XT_R, HB_XT_D>(n, batch, ld, X, bx, Mb, bm, Xo, bo, st);
}

template <bool LOWER, int D>
hipError_t launch_m_d(int64_t n, int64_t batch, int64_t ld, const Tri& T, int q, const double* X,
                      int64_t bx, double* Mb, int64_t bm, hipStream_t st) {
  const int64_t tiles = (n + 3) / 4;
  const int64_t chunks = (bm + D) / D;
  const int64_t work = ((batch + 63) / 64) * tiles * chunks;
  if (work > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((hb_m_kernel<LOWER, D>), dim3((unsigned)work), dim3(kBlock), 0, st, n, batch,
                     ld, T, q, X, bx, Mb, bm, tiles, chunks, work);
  return hipGetLastError();
}

template <bool LOWER>
hipError_t launch_m(int64_t n, int64_t batch, int64_t ld, const Tri& T, int q, const double* X,
                    int64_t bx, double* Mb, int64_t bm, hipStream_t st) {
  if (bm < 4) return launch_m_d<LOWER, 4>(n, batch, ld, T, q, X, bx, Mb, bm, st);
  return launch_m_d<LOWER, 8>(n, batch, ld, T, q, X, bx, Mb, bm, st);
}

template <bool LOWER, int Q, int R, int D>
hipError_t launch_xf_rd(int64_t n, int64_t batch, int64_t ld, const Tri& T, const double* X,
                        int64_t bx, int64_t bm, double* Xo, int64_t bo, hipStream_t st) {
  const int64_t tiles = (n + 4 * R - 1) / (4 * R);
  const int64_t chunks = (bo + D) / D;
  const int64_t work = ((batch + 63) / 64) * tiles * chunks;
  if (work > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((hb_xf_kernel<LOWER, Q, R, D>), dim3((unsigned)work), dim3(kBlock), 0, st,
                     n, batch, ld, T, X, bx, bm, Xo, bo, tiles, chunks, work);
  return hipGetLastError();
}

// The fused step wins while the output band is narrow (measured on the
// 2048 x 2048 sweep factors: 0.57 against 0.75 ms for the first three steps
// of each factor at s = (5, 6)); from band 16 on, the step whose product
// only loads M is faster (band 126: 6.4 against 8.8 ms).
constexpr int64_t kFusedBelow = 16;

template <bool LOWER, int Q>
hipError_t launch_xf(int64_t n, int64_t batch, int64_t ld, const Tri& T, const double* X,
                     int64_t bx, int64_t bm, double* Xo, int64_t bo, hipStream_t st) {
  if (bo < 4) return launch_xf_rd<LOWER, Q, 4, 4>(n, batch, ld, T, X, bx, bm, Xo, bo, st);
  return launch_xf_rd<LOWER, Q, 4, 8>(n, batch, ld, T, X, bx, bm, Xo, bo, st);
}

// One factor: s steps; the result lands in `out`, intermediates alternate
// between `out` and `xw` so that the last step writes `out`.
template <bool LOWER>
hipError_t hb_factor(int64_t n, int64_t batch, int64_t ld, const Tri& T, int q, int s,
                     double* out, double* xw, double* mw, hipStream_t st) {
  const dim3 grid(grid_for(n * batch)), block(kBlock);
  auto buf = [&](int j) { return ((s - j) % 2 == 0) ? out : xw; };
  hipLaunchKernelGGL(hb_init_kernel, grid, block, 0, st, n, batch, ld, T, buf(0));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int j = 0; j < s; ++j) {
    const int64_t bx = band_width(q, j, n);
    const int64_t bm = bx + q < n - 1 ? bx + q : n - 1;
    const int64_t bo = band_width(q, j + 1, n);
    if (bo < kFusedBelow) {  // narrow bands: M formed inside the product
      e = q == 2 ? launch_xf<LOWER, 2>(n, batch, ld, T, buf(j), bx, bm, buf(j + 1), bo, st)
                 : launch_xf<LOWER, 1>(n, batch, ld, T, buf(j), bx, bm, buf(j + 1), bo, st);
    } else {
      e = launch_m<LOWER>(n, batch, ld, T, q, buf(j), bx, mw, bm, st);
      if (e != hipSuccess) return e;
      e = launch_xt<LOWER>(n, batch, ld, buf(j), bx, mw, bm, buf(j + 1), bo, st);
    }
    if (e != hipSuccess) return e;
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

bool ok_ptr(const void* p) { return p != nullptr && reinterpret_cast<uintptr_t>(p) % 8 == 0; }

}  // namespace

int64_t hb_band_width(int kind, int s, int64_t n) { return band_width(kind == 5 ? 2 : 1, s, n); }

}  // namespace bs

extern "C" size_t hb_inverse_band_workspace_bytes(int32_t kind, int64_t n, int64_t batch,
                                                  int64_t ld, int32_t s_L, int32_t s_U) {
  // batch < 2^28: a lane's byte offset 8 s is a 32-bit value
  if ((kind != 3 && kind != 5) || n < 1 || batch < 1 || batch >= (int64_t(1) << 28) ||
      ld < batch || s_L < 0 || s_U < 0 || s_L > 30 || s_U > 30 || ld > (int64_t(1) << 40) / n)
    return (size_t)-1;
  const int64_t K = bs::hb_band_width(kind, s_L > s_U ? s_L : s_U, n);
  // every launch's grid (at most (K + 8) / 8 distance chunks of n / 4 rows
  // per 64 systems) must fit a one-dimensional grid
  const int64_t lim = 0x7fffffff, g1 = (batch + 63) / 64, g2 = (n + 3) / 4, g3 = (K + 8) / 8;
  if (g1 > lim / g2 || g1 * g2 > lim / g3) return (size_t)-1;
  return (size_t)(2 * (K + 1) * n * ld) * sizeof(double);
}

extern "C" int32_t hb_inverse_band(int32_t kind, int64_t n, int64_t batch, int64_t ld,
                                   const void* const diags[5], const double* factors,
                                   int32_t s_L, int32_t s_U, double* XL, double* XU,
                                   void* workspace, size_t ws_bytes, void* stream) {
  const size_t need = hb_inverse_band_workspace_bytes(kind, n, batch, ld, s_L, s_U);
  if (need == (size_t)-1 || diags == nullptr || !bs::ok_ptr(factors) ||
      (XL == nullptr && XU == nullptr))
    return BS_EINVAL;
  if ((XL && !bs::ok_ptr(XL)) || (XU && !bs::ok_ptr(XU))) return BS_EINVAL;
  // U needs A's upper diagonals: a (kind 3) or b (kind 5)
  const void* up = kind == 5 ? diags[4] : diags[3];
  if (XU && !bs::ok_ptr(up)) return BS_EINVAL;
  if (ws_bytes < need) return BS_EWORKSPACE;
  if (!bs::ok_ptr(workspace)) return BS_EINVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return BS_ENODEV;
  const int64_t plane = n * ld;
  const int64_t K = bs::hb_band_width(kind, s_L > s_U ? s_L : s_U, n);
  double* xw = static_cast<double*>(workspace);
  double* mw = xw + (K + 1) * plane;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int q = kind == 5 ? 2 : 1;
  hipError_t e = hipSuccess;
  if (XL) {  // L: unit diagonal; l1 (plane 1 for kind 5, 0 for kind 3), l2 (plane 0)
    const bs::Tri T{nullptr, factors + (kind == 5 ? 1 : 0) * plane,
                    kind == 5 ? factors : nullptr};
    e = bs::hb_factor<true>(n, batch, ld, T, q, s_L, XL, xw, mw, st);
  }
  if (e == hipSuccess && XU) {  // U: u0 (plane 2 / 1), u1 (plane 3 / A's a), u2 = b
    const bs::Tri T{factors + (kind == 5 ? 2 : 1) * plane,
                    kind == 5 ? factors + 3 * plane : static_cast<const double*>(up),
                    kind == 5 ? static_cast<const double*>(up) : nullptr};
    e = bs::hb_factor<false>(n, batch, ld, T, q, s_U, XU, xw, mw, st);
  }
  return e == hipSuccess ? BS_OK : BS_ELAUNCH;
}
