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
// matrices.  Each step is two launches over (row, system): M = 2 I - T X_j,
// then X_{j+1} = X_j M.  Entries are stored by distance from the diagonal:
// plane d of a lower factor holds X[i, i - d] at d*n*ld + i*ld + s, plane d
// of an upper one X[i, i + d]; slots outside the matrix hold 0.
#include "bandsolve.h"
#include "bs_internal.h"

namespace bs {
namespace {

constexpr int kBlock = 256;

struct Tri {  // the factor T: diagonal (null: unit), then q off-diagonals
  const double* dg;
  const double* o1;  // first off-diagonal (l1 below / u1 above)
  const double* o2;  // second off-diagonal (l2 / u2), null when q = 1
};

// T[i, l] for |l - i| <= q on the factor's side of the diagonal (0 outside).
template <bool LOWER>
__device__ inline double tval(const Tri& T, int64_t n, int64_t ld, int64_t i, int64_t l,
                              int64_t s) {
  const int64_t dist = LOWER ? i - l : l - i;
  if (l < 0 || l >= n || dist < 0 || dist > 2) return 0.0;
  const int64_t o = i * ld + s;
  if (dist == 0) return T.dg ? T.dg[o] : 1.0;
  if (dist == 1) return T.o1[o];
  return T.o2 ? T.o2[o] : 0.0;
}

// X[r, c] of a band stored by distance (0 outside the band or the matrix).
template <bool LOWER>
__device__ inline double bval(const double* X, int64_t n, int64_t ld, int64_t band, int64_t r,
                              int64_t c, int64_t s) {
  const int64_t dist = LOWER ? r - c : c - r;
  if (r < 0 || r >= n || c < 0 || c >= n || dist < 0 || dist > band) return 0.0;
  return X[(dist * n + r) * ld + s];
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

// M = 2 I - T X_j (band bm = bx + q): row i of system s per work item.
template <bool LOWER>
__global__ __launch_bounds__(kBlock) void hb_m_kernel(int64_t n, int64_t batch, int64_t ld,
                                                      Tri T, int q, const double* __restrict__ X,
                                                      int64_t bx, double* __restrict__ Mb,
                                                      int64_t bm) {
#pragma clang fp contract(off)
  for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < n * batch;
       w += (int64_t)gridDim.x * kBlock) {
    const int64_t s = w % batch, i = w / batch;
    for (int64_t d = 0; d <= bm; ++d) {
      const int64_t k = LOWER ? i - d : i + d;
      double v = 0.0;
      if (k >= 0 && k < n) {
        double acc = 0.0;  // (T X)[i, k], inner index ascending
        const int64_t l0 = LOWER ? i - q : i, l1 = LOWER ? i : i + q;
        for (int64_t l = l0; l <= l1; ++l) {
          const double t = tval<LOWER>(T, n, ld, i, l, s);
          const double x = bval<LOWER>(X, n, ld, bx, l, k, s);
          if (t != 0.0 && x != 0.0) acc = acc + t * x;
        }
        v = (d == 0 ? 2.0 : 0.0) - acc;
      }
      Mb[(d * n + i) * ld + s] = v;
    }
  }
}

// X_{j+1} = X_j M (band bo = bx + bm): row i of system s per work item.
template <bool LOWER>
__global__ __launch_bounds__(kBlock) void hb_x_kernel(int64_t n, int64_t batch, int64_t ld,
                                                      const double* __restrict__ X, int64_t bx,
                                                      const double* __restrict__ Mb, int64_t bm,
                                                      double* __restrict__ Xo, int64_t bo) {
#pragma clang fp contract(off)
  for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < n * batch;
       w += (int64_t)gridDim.x * kBlock) {
    const int64_t s = w % batch, i = w / batch;
    for (int64_t d = 0; d <= bo; ++d) {
      const int64_t k = LOWER ? i - d : i + d;
      double acc = 0.0;
      if (k >= 0 && k < n) {
        // l between i and k, within bx of i and bm of k, ascending
        const int64_t lo = LOWER ? (k > i - bx ? k : i - bx) : (i > k - bm ? i : k - bm);
        const int64_t hi = LOWER ? (i < k + bm ? i : k + bm) : (k < i + bx ? k : i + bx);
        for (int64_t l = lo; l <= hi; ++l) {
          const double x = bval<LOWER>(X, n, ld, bx, i, l, s);
          const double m = bval<LOWER>(Mb, n, ld, bm, l, k, s);
          if (x != 0.0 && m != 0.0) acc = acc + x * m;
        }
      }
      Xo[(d * n + i) * ld + s] = acc;
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
    hipLaunchKernelGGL((hb_m_kernel<LOWER>), grid, block, 0, st, n, batch, ld, T, q, buf(j), bx,
                       mw, bm);
    hipLaunchKernelGGL((hb_x_kernel<LOWER>), grid, block, 0, st, n, batch, ld, buf(j), bx, mw,
                       bm, buf(j + 1), bo);
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
  if ((kind != 3 && kind != 5) || n < 1 || batch < 1 || ld < batch || s_L < 0 || s_U < 0 ||
      s_L > 30 || s_U > 30 || ld > (int64_t(1) << 40) / n)
    return (size_t)-1;
  const int64_t K = bs::hb_band_width(kind, s_L > s_U ? s_L : s_U, n);
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
