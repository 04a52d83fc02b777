// direct_lane.hip -- NPDM, NTDM, MNPDM, band ILU(0) and band substitution
// with one lane per system (Veneva & Ayriyan, arXiv:1804.09666, Sec. 1-2).
//
// Layout: element (row i, system s) at p[i*ld + s]; lane s walks the rows of
// system s, so each row access of a wave is one contiguous 512-byte segment.
// The forward sweep keeps its recurrence state in registers and streams the
// per-row results that the backward sweep needs (alpha, beta; z goes to x)
// through the caller's workspace.
//
// These kernels evaluate every expression in the bracketed order of the
// sequential recurrences, with IEEE division and without contraction into
// FMAs, so their results are the sequential recurrence's to the last bit.
#include "bs_internal.h"
#include "lane_stream.h"

#pragma clang fp contract(off)

namespace bs {
namespace {

constexpr int kLaneBlock = 64;  // one wave per block: spreads few systems over many CUs

__device__ inline bool bad_pivot(double m) { return !(m != 0.0) || !isfinite(m); }

constexpr int kPF = 8;  // rows in flight per lane (x <= 8 memory operations < 64)

// NPDM: gamma_i = c_i - alpha_{i-2} e_i;  mu_i = (d_i - beta_{i-2} e_i) -
// alpha_{i-1} gamma_i;  alpha_i = (a_i - beta_{i-1} gamma_i) / mu_i;
// beta_i = b_i / mu_i;  z_i = ((y_i - z_{i-2} e_i) - z_{i-1} gamma_i) / mu_i;
// x_i = (z_i - alpha_i x_{i+1}) - beta_i x_{i+2}.
template <typename T>
__global__ __launch_bounds__(kLaneBlock) void npdm_lane_kernel(
    int64_t n, int64_t batch, int64_t ld, const T* __restrict__ E,
    const T* __restrict__ C, const T* __restrict__ D, const T* __restrict__ A,
    const T* __restrict__ B, const T* __restrict__ Y, T* __restrict__ X,
    int32_t* __restrict__ info, T* __restrict__ ws, int64_t lw) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch) return;
  T* al = ws;
  T* be = ws + n * lw;
  T am1 = 0, am2 = 0, bm1 = 0, bm2 = 0, zm1 = 0, zm2 = 0;
  int64_t bad = -1;  // first bad pivot (the sweeps run on; x is then unspecified)
  {
    T re[kPF], rc[kPF], rd[kPF], ra[kPF], rb[kPF], ry[kPF];
    auto fetch = [&](int q, int64_t i) {
      const int64_t o = i * ld + s;
      re[q] = E[o];
      rc[q] = C[o];
      rd[q] = D[o];
      ra[q] = A[o];
      rb[q] = B[o];
      ry[q] = Y[o];
    };
    auto use = [&](int q, int64_t i) {
      const int64_t o = i * ld + s;
      T gamma = 0, mu;
      if (i == 0) {
        mu = rd[q];
      } else if (i == 1) {
        gamma = rc[q];
        mu = rd[q] - am1 * gamma;
      } else {
        gamma = rc[q] - am2 * re[q];
        mu = (rd[q] - bm2 * re[q]) - am1 * gamma;
      }
      if (bad < 0 && bad_pivot(mu)) bad = i;
      T ali = 0, bei = 0, zi;
      if (i <= n - 2) ali = (i == 0) ? ra[q] / mu : (ra[q] - bm1 * gamma) / mu;
      if (i <= n - 3) bei = rb[q] / mu;
      if (i == 0)
        zi = ry[q] / mu;
      else if (i == 1)
        zi = (ry[q] - zm1 * gamma) / mu;
      else
        zi = ((ry[q] - zm2 * re[q]) - zm1 * gamma) / mu;
      al[i * lw + s] = ali;
      be[i * lw + s] = bei;
      X[o] = zi;
      am2 = am1; am1 = ali;
      bm2 = bm1; bm1 = bei;
      zm2 = zm1; zm1 = zi;
    };
    stream_rows<kPF, false>(n, fetch, use);
  }
  {
    T rz[kPF], ral[kPF], rbe[kPF];
    T xp1 = 0, xp2 = 0;  // x_{i+1}, x_{i+2}
    auto fetch = [&](int q, int64_t i) {
      rz[q] = X[i * ld + s];
      ral[q] = al[i * lw + s];
      rbe[q] = be[i * lw + s];
    };
    auto use = [&](int q, int64_t i) {
      T xi;
      if (i == n - 1)
        xi = rz[q];
      else if (i == n - 2)
        xi = rz[q] - ral[q] * xp1;
      else
        xi = (rz[q] - ral[q] * xp1) - rbe[q] * xp2;
      X[i * ld + s] = xi;
      xp2 = xp1;
      xp1 = xi;
    };
    stream_rows<kPF, true>(n, fetch, use);
  }
  info[s] = bad < 0 ? 0 : (int32_t)(bad + 1);
}

// NTDM (Thomas): mu_i = d_i - alpha_{i-1} c_i;  alpha_i = a_i / mu_i;
// z_i = (y_i - z_{i-1} c_i) / mu_i;  x_i = z_i - alpha_i x_{i+1}.
template <typename T>
__global__ __launch_bounds__(kLaneBlock) void ntdm_lane_kernel(
    int64_t n, int64_t batch, int64_t ld, const T* __restrict__ C,
    const T* __restrict__ D, const T* __restrict__ A, const T* __restrict__ Y,
    T* __restrict__ X, int32_t* __restrict__ info, T* __restrict__ ws,
    int64_t lw) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch) return;
  T am1 = 0, zm1 = 0;
  int64_t bad = -1;
  {
    T rc[kPF], rd[kPF], ra[kPF], ry[kPF];
    auto fetch = [&](int q, int64_t i) {
      const int64_t o = i * ld + s;
      rc[q] = C[o];
      rd[q] = D[o];
      ra[q] = A[o];
      ry[q] = Y[o];
    };
    auto use = [&](int q, int64_t i) {
      T mu, ci = 0;
      if (i == 0) {
        mu = rd[q];
      } else {
        ci = rc[q];
        mu = rd[q] - am1 * ci;
      }
      if (bad < 0 && bad_pivot(mu)) bad = i;
      T ali = 0;
      if (i <= n - 2) ali = ra[q] / mu;
      const T zi = (i == 0) ? ry[q] / mu : (ry[q] - zm1 * ci) / mu;
      ws[i * lw + s] = ali;
      X[i * ld + s] = zi;
      am1 = ali;
      zm1 = zi;
    };
    stream_rows<kPF, false>(n, fetch, use);
  }
  {
    T rz[kPF], ral[kPF];
    T xp1 = 0;
    auto fetch = [&](int q, int64_t i) {
      rz[q] = X[i * ld + s];
      ral[q] = ws[i * lw + s];
    };
    auto use = [&](int q, int64_t i) {
      const T xi = (i == n - 1) ? rz[q] : rz[q] - ral[q] * xp1;
      X[i * ld + s] = xi;
      xp1 = xi;
    };
    stream_rows<kPF, true>(n, fetch, use);
  }
  info[s] = bad < 0 ? 0 : (int32_t)(bad + 1);
}

// MNPDM: NPDM with the products of absent outer entries skipped.  The list of
// system s is (outer_row[k*ld+s], oe[k*ld+s], ob[k*ld+s]), k < kmax, strictly
// ascending rows, -1 terminated.  e of rows < 2 and b of rows > n-3 lie
// outside the matrix and are ignored, as are zero values.
__global__ __launch_bounds__(kLaneBlock) void mnpdm_lane_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ C,
    const double* __restrict__ D, const double* __restrict__ A, int32_t kmax,
    const int32_t* __restrict__ orow, const double* __restrict__ oe,
    const double* __restrict__ ob, const double* __restrict__ Y,
    double* __restrict__ X, int32_t* __restrict__ info,
    double* __restrict__ ws, int64_t lw) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch) return;
  // validate the list first: strictly ascending rows in [0, n), then -1s
  {
    int64_t prev = -1;
    bool ended = false;
    for (int32_t k = 0; k < kmax; ++k) {
      const int32_t r = orow[(int64_t)k * ld + s];
      if (r < 0) {
        ended = true;
        continue;
      }
      if (ended || r >= n || r <= prev) {
        info[s] = -3;
        return;
      }
      prev = r;
    }
  }
  double* al = ws;
  double* be = ws + n * lw;
  double am1 = 0, am2 = 0, bm1 = 0, bm2 = 0, zm1 = 0, zm2 = 0;
  bool hb1 = false, hb2 = false;  // beta_{i-1}, beta_{i-2} present
  int32_t q = 0;
  int32_t nr = (kmax > 0) ? orow[s] : -1;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t o = i * ld + s;
    double ei = 0.0, bi = 0.0;
    if (nr == i) {
      const int64_t qo = (int64_t)q * ld + s;
      ei = oe[qo];
      bi = ob[qo];
      ++q;
      nr = (q < kmax) ? orow[(int64_t)q * ld + s] : -1;
    }
    const bool he = (i >= 2) && (ei != 0.0);
    const bool hb = (i <= n - 3) && (bi != 0.0);
    double gamma = 0.0, mu;
    if (i == 0) {
      mu = D[o];
    } else {
      gamma = C[o];
      if (he) gamma = C[o] - am2 * ei;
      mu = D[o];
      if (he && hb2) mu = D[o] - bm2 * ei;
      mu = mu - am1 * gamma;
    }
    if (bad_pivot(mu)) {
      info[s] = (int32_t)(i + 1);
      return;
    }
    double ali = 0.0, bei = 0.0, zi;
    if (i <= n - 2) ali = (i >= 1 && hb1) ? (A[o] - bm1 * gamma) / mu : A[o] / mu;
    if (hb) bei = bi / mu;
    if (i == 0)
      zi = Y[o] / mu;
    else if (he)
      zi = ((Y[o] - zm2 * ei) - zm1 * gamma) / mu;
    else
      zi = (Y[o] - zm1 * gamma) / mu;
    al[i * lw + s] = ali;
    be[i * lw + s] = hb ? bei : 0.0;
    X[o] = zi;
    am2 = am1; am1 = ali;
    bm2 = bm1; bm1 = bei;
    hb2 = hb1; hb1 = hb;
    zm2 = zm1; zm1 = zi;
  }
  double xp1 = 0, xp2 = 0;
  for (int64_t i = n - 1; i >= 0; --i) {
    const int64_t o = i * ld + s;
    const double zi = X[o];
    double xi;
    if (i == n - 1) {
      xi = zi;
    } else {
      const double bei = be[i * lw + s];
      xi = zi - al[i * lw + s] * xp1;
      if (bei != 0.0) xi = xi - bei * xp2;
    }
    X[o] = xi;
    xp2 = xp1;
    xp1 = xi;
  }
  info[s] = 0;
}

// Band Doolittle ILU(0): l2_i = e_i / u0_{i-2};  l1_i = (c_i - l2_i u1_{i-2})
// / u0_{i-1};  u0_i = (d_i - l2_i u2_{i-2}) - l1_i u1_{i-1};
// u1_i = a_i - l1_i u2_{i-1};  u2_i = b_i.
template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void factor_lane_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ E,
    const double* __restrict__ C, const double* __restrict__ D,
    const double* __restrict__ A, const double* __restrict__ B,
    double* __restrict__ F, int64_t fld, int32_t* __restrict__ info) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch) return;
  const int64_t plane = n * fld;
  double* L2 = (KIND == 5) ? F : nullptr;
  double* L1 = (KIND == 5) ? F + plane : F;
  double* U0 = (KIND == 5) ? F + 2 * plane : F + plane;
  double* U1 = (KIND == 5) ? F + 3 * plane : nullptr;
  double re[kPF], rc[kPF], rd[kPF], ra[kPF], rb[kPF];
  auto fetch = [&](int q, int64_t i) {
    const int64_t o = i * ld + s;
    if (KIND == 5) re[q] = E[o];
    rc[q] = C[o];
    rd[q] = D[o];
    ra[q] = A[o];
    if (KIND == 5) rb[q] = B[o];
  };
  double u0m1 = 0, u0m2 = 0, u1m1 = 0, u1m2 = 0, u2m1 = 0, u2m2 = 0;
  int64_t bad = -1;  // first bad pivot (the sweep runs on; later factors unspecified)
  auto use = [&](int q, int64_t i) {
    // corner slots (e_0, e_1, c_0, a_{n-1}, b_{n-2}, b_{n-1}) are never used
    double l2 = 0.0, l1 = 0.0, u0, u1 = 0.0, u2 = 0.0;
    if (KIND == 5 && i >= 2) l2 = re[q] / u0m2;
    if (i == 1) l1 = rc[q] / u0m1;
    if (i >= 2) l1 = (KIND == 5) ? (rc[q] - l2 * u1m2) / u0m1 : rc[q] / u0m1;
    if (i == 0)
      u0 = rd[q];
    else if (i == 1 || KIND == 3)
      u0 = rd[q] - l1 * u1m1;
    else
      u0 = (rd[q] - l2 * u2m2) - l1 * u1m1;
    if (bad < 0 && bad_pivot(u0)) bad = i;
    if (i <= n - 2) u1 = (i == 0 || KIND == 3) ? ra[q] : ra[q] - l1 * u2m1;
    if (KIND == 5 && i <= n - 3) u2 = rb[q];
    const int64_t fo = i * fld + s;
    if (KIND == 5) {
      L2[fo] = l2;
      U1[fo] = u1;
    }
    L1[fo] = l1;
    U0[fo] = u0;
    u0m2 = u0m1; u0m1 = u0;
    u1m2 = u1m1; u1m1 = u1;
    u2m2 = u2m1; u2m1 = u2;
  };
  stream_rows<kPF, false>(n, fetch, use);
  info[s] = bad < 0 ? 0 : (int32_t)(bad + 1);
}

// Substitution with the band factors: z_i = (y_i - l1_i z_{i-1}) - l2_i z_{i-2}
// (z kept in x), then x_i = ((z_i - u1_i x_{i+1}) - u2_i x_{i+2}) / u0_i.
template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void subst_lane_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ Aa,
    const double* __restrict__ B, const double* __restrict__ F,
    const double* __restrict__ Y, double* __restrict__ X,
    int32_t* __restrict__ info) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch) return;
  const int64_t plane = n * ld;
  const double* L2 = (KIND == 5) ? F : nullptr;
  const double* L1 = (KIND == 5) ? F + plane : F;
  const double* U0 = (KIND == 5) ? F + 2 * plane : F + plane;
  const double* U1 = (KIND == 5) ? F + 3 * plane : Aa;  // TD: u1 = a
  {
    double ry[kPF], rl1[kPF], rl2[kPF];
    double zm1 = 0, zm2 = 0;
    auto fetch = [&](int q, int64_t i) {
      const int64_t o = i * ld + s;
      ry[q] = Y[o];
      rl1[q] = L1[o];
      if (KIND == 5) rl2[q] = L2[o];
    };
    auto use = [&](int q, int64_t i) {
      double t = ry[q];
      if (i >= 1) t = t - rl1[q] * zm1;
      if (KIND == 5 && i >= 2) t = t - rl2[q] * zm2;
      X[i * ld + s] = t;
      zm2 = zm1;
      zm1 = t;
    };
    stream_rows<kPF, false>(n, fetch, use);
  }
  {
    double rz[kPF], ru1[kPF], ru2[kPF], ru0[kPF];
    double xp1 = 0, xp2 = 0;
    auto fetch = [&](int q, int64_t i) {
      const int64_t o = i * ld + s;
      rz[q] = X[o];
      ru1[q] = U1[o];
      if (KIND == 5) ru2[q] = B[o];
      ru0[q] = U0[o];
    };
    auto use = [&](int q, int64_t i) {
      double t = rz[q];
      if (i + 1 < n) t = t - ru1[q] * xp1;
      if (KIND == 5 && i + 2 < n) t = t - ru2[q] * xp2;
      const double xi = t / ru0[q];
      X[i * ld + s] = xi;
      xp2 = xp1;
      xp1 = xi;
    };
    stream_rows<kPF, true>(n, fetch, use);
  }
  info[s] = 0;
}

inline dim3 lane_grid(int64_t batch) {
  return dim3((unsigned)((batch + kLaneBlock - 1) / kLaneBlock));
}

}  // namespace

hipError_t launch_npdm_lane(int64_t n, int64_t batch, int64_t ld, Diags A,
                            const double* y, double* x, int32_t* info,
                            double* ws, hipStream_t st) {
  hipLaunchKernelGGL(npdm_lane_kernel<double>, lane_grid(batch),
                     dim3(kLaneBlock), 0, st, n, batch, ld, A.e, A.c, A.d, A.a,
                     A.b, y, x, info, ws, ws_ld(batch));
  return hipGetLastError();
}

hipError_t launch_ntdm_lane(int64_t n, int64_t batch, int64_t ld, Diags A,
                            const double* y, double* x, int32_t* info,
                            double* ws, hipStream_t st) {
  hipLaunchKernelGGL(ntdm_lane_kernel<double>, lane_grid(batch),
                     dim3(kLaneBlock), 0, st, n, batch, ld, A.c, A.d, A.a, y,
                     x, info, ws, ws_ld(batch));
  return hipGetLastError();
}

hipError_t launch_mnpdm_lane(int64_t n, int64_t batch, int64_t ld, Diags A,
                             int32_t kmax, const int32_t* orow,
                             const double* oe, const double* ob,
                             const double* y, double* x, int32_t* info,
                             double* ws, hipStream_t st) {
  hipLaunchKernelGGL(mnpdm_lane_kernel, lane_grid(batch), dim3(kLaneBlock), 0,
                     st, n, batch, ld, A.c, A.d, A.a, kmax, orow, oe, ob, y, x,
                     info, ws, ws_ld(batch));
  return hipGetLastError();
}

hipError_t launch_factor_lane(int kind, int64_t n, int64_t batch, int64_t ld,
                              Diags A, double* factors, int64_t fld,
                              int32_t* info, hipStream_t st) {
  if (kind == 5)
    hipLaunchKernelGGL(factor_lane_kernel<5>, lane_grid(batch),
                       dim3(kLaneBlock), 0, st, n, batch, ld, A.e, A.c, A.d,
                       A.a, A.b, factors, fld, info);
  else
    hipLaunchKernelGGL(factor_lane_kernel<3>, lane_grid(batch),
                       dim3(kLaneBlock), 0, st, n, batch, ld, A.e, A.c, A.d,
                       A.a, A.b, factors, fld, info);
  return hipGetLastError();
}

hipError_t launch_subst_lane(int kind, int64_t n, int64_t batch, int64_t ld,
                             Diags A, const double* factors, const double* y,
                             double* x, int32_t* info, hipStream_t st) {
  if (kind == 5)
    hipLaunchKernelGGL(subst_lane_kernel<5>, lane_grid(batch),
                       dim3(kLaneBlock), 0, st, n, batch, ld, A.a, A.b,
                       factors, y, x, info);
  else
    hipLaunchKernelGGL(subst_lane_kernel<3>, lane_grid(batch),
                       dim3(kLaneBlock), 0, st, n, batch, ld, A.a, A.b,
                       factors, y, x, info);
  return hipGetLastError();
}

}  // namespace bs
