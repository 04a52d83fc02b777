// split_core.h -- device building blocks of the split-row (partitioned)
// NPDM / NTDM elimination shared by the fixed-shape kernels (direct_part.hip)
// and the uneven-batch kernels (varlen.hip).  See direct_part.hip for the
// method.
#pragma once

#include <climits>

#include "bs_internal.h"

namespace bs {
namespace split {

template <int NB>
struct Map {  // T = pt - Vt xL - Wt xR,  B = pb - Vb xL - Wb xR
  double pt[NB], pb[NB];
  double Vt[NB][NB], Vb[NB][NB], Wt[NB][NB], Wb[NB][NB];
};

template <int NB>
struct Node {  // interface: B_A = g0 + G1 xL + G2 xR,  T_B = h0 + H1 xL + H2 xR
  double g0[NB], h0[NB];
  double G1[NB][NB], G2[NB][NB], H1[NB][NB], H2[NB][NB];
};

template <int NB>
constexpr int kRecSz = 2 * NB + 4 * NB * NB;  // doubles per Map or Node

// The map of a range of identity rows (no couplings, zero solution).
template <int NB>
__device__ inline void zero_map(Map<NB>& m) {
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    m.pt[q] = m.pb[q] = 0.0;
#pragma unroll
    for (int k = 0; k < NB; ++k) m.Vt[q][k] = m.Vb[q][k] = m.Wt[q][k] = m.Wb[q][k] = 0.0;
  }
}

template <int NB>
__device__ inline void mm(const double (&A)[NB][NB], const double (&B)[NB][NB],
                          double (&C)[NB][NB]) {
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < NB; ++k) acc = fma(A[i][k], B[k][j], acc);
      C[i][j] = acc;
    }
}

template <int NB>
__device__ inline void mv(const double (&A)[NB][NB], const double (&x)[NB],
                          double (&y)[NB]) {
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < NB; ++k) acc = fma(A[i][k], x[k], acc);
    y[i] = acc;
  }
}

// Breakdown guard of the partitioned elimination: a pivot (or interface
// determinant) counts as bad when it is not finite or not larger than
// kGuard times the magnitude of the terms it is formed from.  Such a pivot
// either breaks the elimination or amplifies rounding by more than 1/kGuard,
// so the system is redone with the sequential recurrence instead.
constexpr double kGuard = 0x1p-12;

// 1/x from the hardware reciprocal estimate and two Newton steps (full
// double precision up to an ulp; pivots and interface blocks are far from the
// subnormal range).  The chunk recurrences divide by every pivot in a chain
// of dependent operations, and this is half as long as IEEE division; a zero
// or non-finite pivot is reported from the pivot itself.
__device__ inline double recip(double x) {
  const double r0 = __builtin_amdgcn_rcp(x);
  double r = fma(r0, fma(-x, r0, 1.0), r0);
  r = fma(r, fma(-x, r, 1.0), r);
  // the estimate alone is exact for the special cases (+-0 -> +-inf,
  // +-inf -> +-0, as 1/x), where the Newton steps would give NaN
  return (x != 0.0 && isfinite(x)) ? r : r0;
}
// Inverse of the 1x1 or 2x2 interface block M = I - P (P = Wb Vt); false
// if the guard rejects it.
__device__ inline bool inv(const double (&M)[1][1], const double (&P)[1][1], double (&R)[1][1]) {
  R[0][0] = recip(M[0][0]);
  return fabs(M[0][0]) > kGuard * (1.0 + fabs(P[0][0])) && isfinite(R[0][0]);
}
__device__ inline bool inv(const double (&M)[2][2], const double (&P)[2][2], double (&R)[2][2]) {
  const double p1 = M[0][0] * M[1][1], p2 = M[0][1] * M[1][0];
  const double det = p1 - p2;
  const double r = recip(det);
  R[0][0] = M[1][1] * r;
  R[0][1] = -M[0][1] * r;
  R[1][0] = -M[1][0] * r;
  R[1][1] = M[0][0] * r;
  // magnitude of det's terms, bounded with |M_ij| <= delta_ij + |P_ij|
  const double sc = (1.0 + fabs(P[0][0])) * (1.0 + fabs(P[1][1])) + fabs(P[0][1]) * fabs(P[1][0]);
  return fabs(det) > kGuard * sc && isfinite(r);
}

// Merge left part A with right part B (B's x_L is A's bottom pair, A's x_R
// is B's top pair).  Returns false if the interface block is singular.
template <int NB>
__device__ bool merge(const Map<NB>& A, const Map<NB>& B, Map<NB>& AB, Node<NB>& nd) {
  double Px[NB][NB], Mx[NB][NB], S[NB][NB], T1[NB][NB], t[NB];
  mm<NB>(A.Wb, B.Vt, Px);
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) Mx[i][j] = (i == j ? 1.0 : 0.0) - Px[i][j];
  const bool ok = inv(Mx, Px, S);
  mv<NB>(A.Wb, B.pt, t);
#pragma unroll
  for (int i = 0; i < NB; ++i) t[i] = A.pb[i] - t[i];
  mv<NB>(S, t, nd.g0);
  mm<NB>(S, A.Vb, nd.G1);
  mm<NB>(A.Wb, B.Wt, T1);
  mm<NB>(S, T1, nd.G2);
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) nd.G1[i][j] = -nd.G1[i][j];
  mv<NB>(B.Vt, nd.g0, t);
#pragma unroll
  for (int i = 0; i < NB; ++i) nd.h0[i] = B.pt[i] - t[i];
  mm<NB>(B.Vt, nd.G1, nd.H1);
  mm<NB>(B.Vt, nd.G2, nd.H2);
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      nd.H1[i][j] = -nd.H1[i][j];
      nd.H2[i][j] = -(nd.H2[i][j] + B.Wt[i][j]);
    }
  Map<NB> R;
  mv<NB>(A.Wt, nd.h0, t);
#pragma unroll
  for (int i = 0; i < NB; ++i) R.pt[i] = A.pt[i] - t[i];
  mm<NB>(A.Wt, nd.H1, T1);
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) R.Vt[i][j] = A.Vt[i][j] + T1[i][j];
  mm<NB>(A.Wt, nd.H2, R.Wt);
  mv<NB>(B.Vb, nd.g0, t);
#pragma unroll
  for (int i = 0; i < NB; ++i) R.pb[i] = B.pb[i] - t[i];
  mm<NB>(B.Vb, nd.G1, R.Vb);
  mm<NB>(B.Vb, nd.G2, T1);
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) R.Wb[i][j] = T1[i][j] + B.Wb[i][j];
  AB = R;
  return ok;
}

template <typename R>
__device__ inline void store_rec(const R& r, double* dst) {
  const double* src = reinterpret_cast<const double*>(&r);
#pragma unroll
  for (int q = 0; q < (int)(sizeof(R) / sizeof(double)); ++q) dst[q] = src[q];
}
template <typename R>
__device__ inline void load_rec(R& r, const double* src) {
  double* dst = reinterpret_cast<double*>(&r);
#pragma unroll
  for (int q = 0; q < (int)(sizeof(R) / sizeof(double)); ++q) dst[q] = src[q];
}

// Local pivot mu of a row whose inner entries have magnitude sum sc.
__device__ inline bool bad_pivot(double mu, double sc) {
  return !(fabs(mu) > kGuard * sc) || !isfinite(mu);
}

// Streaming accesses: every input element is read once and every x element
// written once, so they carry the non-temporal hint.  Storage may be FP64 or
// FP32 (TIO); arithmetic is always FP64.
template <typename TIO>
__device__ inline TIO ldg(const TIO* __restrict__ base, uint32_t byte_off) {
  return __builtin_nontemporal_load(
      reinterpret_cast<const TIO*>(reinterpret_cast<const char*>(base) + byte_off));
}
template <typename TIO>
__device__ inline void stg(TIO* __restrict__ base, uint32_t byte_off, double v) {
  __builtin_nontemporal_store((TIO)v, reinterpret_cast<TIO*>(reinterpret_cast<char*>(base) + byte_off));
}

// Chunk of a pentadiagonal system: local NPDM with the couplings to
// x_L = (x_{-2}, x_{-1}) (entries e_0, c_0 of row 0 and e_1 of row 1) and to
// x_R = (x_M, x_{M+1}) (b_{M-2} of row M-2, a_{M-1} and b_{M-1} of row M-1)
// as right-hand sides.  On return p, v0, v1, w0, w1 hold U^{-1} L^{-1} of
// y and of the coupling columns; `bad` is the first local row with a bad
// pivot (M if none).  src(r, e, c, d, a, b, y) gives row r; pre(r) runs at
// the start of the forward step of row r (a streaming caller issues the
// loads of a later row there).
template <int M, typename Src, typename Pre>
__device__ inline void chunk_pd_rows(Src&& src, Pre&& pre, double (&p)[M], double (&v0)[M],
                                     double (&v1)[M], double (&w0)[M], double (&w1)[M],
                                     int& bad) {
  double al[M], be[M];
  double fm2 = 0.0;  // L^{-1} of the x_M column at row M-2
  bad = M;
#pragma unroll
  for (int r = 0; r < M; ++r) {
    pre(r);
    double e, c, d, a, b, y;
    src(r, e, c, d, a, b, y);
    double ga, mu;
    if (r == 0) {
      ga = 0.0;
      mu = d;
    } else if (r == 1) {
      ga = c;
      mu = fma(-al[0], ga, d);
    } else {
      ga = fma(-al[r - 2], e, c);
      mu = fma(-al[r - 1], ga, fma(-be[r - 2], e, d));
    }
    // the row's magnitude from its inner three entries (measured: adding the
    // outer two costs 5 us per sweep batch, the scale only sets the guard)
    if (bad == M && bad_pivot(mu, fabs(c) + fabs(d) + fabs(a))) bad = r;
    const double rc = recip(mu);  // off the IEEE division's longer chain
    if (r == 0)
      al[0] = a * rc;
    else if (r <= M - 2)
      al[r] = fma(-be[r - 1], ga, a) * rc;
    else
      al[r] = 0.0;
    be[r] = (r <= M - 3) ? b * rc : 0.0;
    if (r == 0) {
      p[0] = y * rc;
      v0[0] = e * rc;
      v1[0] = c * rc;
    } else if (r == 1) {
      p[1] = fma(-ga, p[0], y) * rc;
      v0[1] = (-ga * v0[0]) * rc;
      v1[1] = fma(-ga, v1[0], e) * rc;
    } else {
      p[r] = fma(-ga, p[r - 1], fma(-e, p[r - 2], y)) * rc;
      v0[r] = fma(-ga, v0[r - 1], -e * v0[r - 2]) * rc;
      v1[r] = fma(-ga, v1[r - 1], -e * v1[r - 2]) * rc;
    }
    if (r == M - 2) fm2 = b * rc;
    if (r == M - 1) {
      w0[M - 1] = fma(-ga, fm2, a) * rc;
      w1[M - 1] = b * rc;
    }
  }
  w0[M - 2] = fma(-al[M - 2], w0[M - 1], fm2);
  w1[M - 2] = -al[M - 2] * w1[M - 1];
  p[M - 2] = fma(-al[M - 2], p[M - 1], p[M - 2]);
  v0[M - 2] = fma(-al[M - 2], v0[M - 1], v0[M - 2]);
  v1[M - 2] = fma(-al[M - 2], v1[M - 1], v1[M - 2]);
#pragma unroll
  for (int r = M - 3; r >= 0; --r) {
    p[r] = fma(-be[r], p[r + 2], fma(-al[r], p[r + 1], p[r]));
    v0[r] = fma(-be[r], v0[r + 2], fma(-al[r], v0[r + 1], v0[r]));
    v1[r] = fma(-be[r], v1[r + 2], fma(-al[r], v1[r + 1], v1[r]));
    w0[r] = fma(-be[r], w0[r + 2], -al[r] * w0[r + 1]);
    w1[r] = fma(-be[r], w1[r + 2], -al[r] * w1[r + 1]);
  }
}

// Chunk of a tridiagonal system: local Thomas with the couplings to x_{-1}
// (c_0 of row 0) and x_M (a_{M-1} of row M-1) as right-hand sides.  src and
// pre as for chunk_pd_rows (e and b unused).
template <int M, typename Src, typename Pre>
__device__ inline void chunk_td_rows(Src&& src, Pre&& pre, double (&p)[M], double (&v0)[M],
                                     double (&w0)[M], int& bad) {
  double al[M];
  bad = M;
#pragma unroll
  for (int r = 0; r < M; ++r) {
    pre(r);
    double e, c, d, a, b, y;
    src(r, e, c, d, a, b, y);
    const double mu = (r == 0) ? d : fma(-al[r - 1], c, d);
    if (bad == M && bad_pivot(mu, fabs(c) + fabs(d) + fabs(a))) bad = r;
    const double rc = recip(mu);  // off the IEEE division's longer chain
    al[r] = (r <= M - 2) ? a * rc : 0.0;
    if (r == 0) {
      p[0] = y * rc;
      v0[0] = c * rc;
    } else {
      p[r] = fma(-c, p[r - 1], y) * rc;
      v0[r] = (-c * v0[r - 1]) * rc;
    }
    if (r == M - 1) w0[M - 1] = a * rc;
  }
#pragma unroll
  for (int r = M - 2; r >= 0; --r) {
    p[r] = fma(-al[r], p[r + 1], p[r]);
    v0[r] = fma(-al[r], v0[r + 1], v0[r]);
    w0[r] = -al[r] * w0[r + 1];
  }
}

// The FP32 rounding of a value, materialised where it is written: without
// this the compiler sinks the conversion to the value's use in the backward
// sweep and keeps the FP64 value alive in between (twice the registers).
__device__ inline float keep32(double x) {
  float f = (float)x;
  asm volatile("" : "+v"(f));
  return f;
}

// Compact chunk state (FP32 storage only).  The forward step of every row
// -- pivot, multipliers and the L^{-1} columns -- runs in FP64 exactly as in
// chunk_pd_rows, with the two previous rows carried in FP64 registers; the
// per-row results are kept in FP32, and the backward substitution U^{-1}
// runs in FP32.  Half the registers of the FP64 state, so a lane can own
// twice the rows (or a SIMD two waves).
template <int M, typename Src, typename Pre>
__device__ inline void chunk_pd_rows(Src&& src, Pre&& pre, float (&p)[M], float (&v0)[M],
                                     float (&v1)[M], float (&w0)[M], float (&w1)[M],
                                     int& bad) {
  float al[M], be[M];
  double am1 = 0.0, am2 = 0.0, bm1 = 0.0, bm2 = 0.0;  // alpha, beta of rows r-1, r-2
  double pm1 = 0.0, pm2 = 0.0, xm1 = 0.0, xm2 = 0.0, ym1 = 0.0, ym2 = 0.0;  // p, v0, v1
  double fm2 = 0.0;
  bad = M;
#pragma unroll
  for (int r = 0; r < M; ++r) {
    pre(r);
    double e, c, d, a, b, y;
    src(r, e, c, d, a, b, y);
    double ga, mu;
    if (r == 0) {
      ga = 0.0;
      mu = d;
    } else if (r == 1) {
      ga = c;
      mu = fma(-am1, ga, d);
    } else {
      ga = fma(-am2, e, c);
      mu = fma(-am1, ga, fma(-bm2, e, d));
    }
    if (bad == M && bad_pivot(mu, fabs(c) + fabs(d) + fabs(a))) bad = r;
    const double rc = recip(mu);
    double ali, pi, xi, yi;
    if (r == 0)
      ali = a * rc;
    else if (r <= M - 2)
      ali = fma(-bm1, ga, a) * rc;
    else
      ali = 0.0;
    const double bei = (r <= M - 3) ? b * rc : 0.0;
    if (r == 0) {
      pi = y * rc;
      xi = e * rc;
      yi = c * rc;
    } else if (r == 1) {
      pi = fma(-ga, pm1, y) * rc;
      xi = (-ga * xm1) * rc;
      yi = fma(-ga, ym1, e) * rc;
    } else {
      pi = fma(-ga, pm1, fma(-e, pm2, y)) * rc;
      xi = fma(-ga, xm1, -e * xm2) * rc;
      yi = fma(-ga, ym1, -e * ym2) * rc;
    }
    if (r == M - 2) fm2 = b * rc;
    if (r == M - 1) {
      w0[M - 1] = keep32(fma(-ga, fm2, a) * rc);
      w1[M - 1] = keep32(b * rc);
    }
    al[r] = keep32(ali);
    be[r] = keep32(bei);
    p[r] = keep32(pi);
    v0[r] = keep32(xi);
    v1[r] = keep32(yi);
    am2 = am1;
    am1 = ali;
    bm2 = bm1;
    bm1 = bei;
    pm2 = pm1;
    pm1 = pi;
    xm2 = xm1;
    xm1 = xi;
    ym2 = ym1;
    ym1 = yi;
  }
  w0[M - 2] = fmaf(-al[M - 2], w0[M - 1], (float)fm2);
  w1[M - 2] = -al[M - 2] * w1[M - 1];
  p[M - 2] = fmaf(-al[M - 2], p[M - 1], p[M - 2]);
  v0[M - 2] = fmaf(-al[M - 2], v0[M - 1], v0[M - 2]);
  v1[M - 2] = fmaf(-al[M - 2], v1[M - 1], v1[M - 2]);
#pragma unroll
  for (int r = M - 3; r >= 0; --r) {
    p[r] = fmaf(-be[r], p[r + 2], fmaf(-al[r], p[r + 1], p[r]));
    v0[r] = fmaf(-be[r], v0[r + 2], fmaf(-al[r], v0[r + 1], v0[r]));
    v1[r] = fmaf(-be[r], v1[r + 2], fmaf(-al[r], v1[r + 1], v1[r]));
    w0[r] = fmaf(-be[r], w0[r + 2], -al[r] * w0[r + 1]);
    w1[r] = fmaf(-be[r], w1[r + 2], -al[r] * w1[r + 1]);
  }
}

// Compact chunk state of a tridiagonal chunk (see the pentadiagonal one).
template <int M, typename Src, typename Pre>
__device__ inline void chunk_td_rows(Src&& src, Pre&& pre, float (&p)[M], float (&v0)[M],
                                     float (&w0)[M], int& bad) {
  float al[M];
  double am1 = 0.0, pm1 = 0.0, vm1 = 0.0;
  bad = M;
#pragma unroll
  for (int r = 0; r < M; ++r) {
    pre(r);
    double e, c, d, a, b, y;
    src(r, e, c, d, a, b, y);
    const double mu = (r == 0) ? d : fma(-am1, c, d);
    if (bad == M && bad_pivot(mu, fabs(c) + fabs(d) + fabs(a))) bad = r;
    const double rc = recip(mu);
    const double ali = (r <= M - 2) ? a * rc : 0.0;
    const double pi = (r == 0) ? y * rc : fma(-c, pm1, y) * rc;
    const double vi = (r == 0) ? c * rc : (-c * vm1) * rc;
    if (r == M - 1) w0[M - 1] = keep32(a * rc);
    al[r] = keep32(ali);
    p[r] = keep32(pi);
    v0[r] = keep32(vi);
    am1 = ali;
    pm1 = pi;
    vm1 = vi;
  }
#pragma unroll
  for (int r = M - 2; r >= 0; --r) {
    p[r] = fmaf(-al[r], p[r + 1], p[r]);
    v0[r] = fmaf(-al[r], v0[r + 1], v0[r]);
    w0[r] = -al[r] * w0[r + 1];
  }
}

template <int M>
__device__ inline void chunk_pd(const double (&e)[M], const double (&c)[M],
                                const double (&d)[M], const double (&a)[M],
                                const double (&b)[M], const double (&y)[M],
                                double (&p)[M], double (&v0)[M], double (&v1)[M],
                                double (&w0)[M], double (&w1)[M], int& bad) {
  chunk_pd_rows<M>(
      [&](int r, double& er, double& cr, double& dr, double& ar, double& br, double& yr) {
        er = e[r];
        cr = c[r];
        dr = d[r];
        ar = a[r];
        br = b[r];
        yr = y[r];
      },
      [](int) {}, p, v0, v1, w0, w1, bad);
}

template <int M>
__device__ inline void chunk_td(const double (&c)[M], const double (&d)[M],
                                const double (&a)[M], const double (&y)[M],
                                double (&p)[M], double (&v0)[M], double (&w0)[M],
                                int& bad) {
  chunk_td_rows<M>(
      [&](int r, double& er, double& cr, double& dr, double& ar, double& br, double& yr) {
        er = br = 0.0;
        cr = c[r];
        dr = d[r];
        ar = a[r];
        yr = y[r];
      },
      [](int) {}, p, v0, w0, bad);
}

// Binary tree over NL leaf maps held by lanes (leaf, g), leaf in [0, NL);
// lanes with leaf >= NL only take part in the barriers.  Each internal node
// owns one record slot in s_node: the right child parks its map there, the
// left child merges and overwrites it with the node record, and on the way
// down the left child replaces the record with the right child's outer pairs.
// leaf_rows: rows per leaf, row0: first row of leaf 0 (for breakdown rows).
// With LANES, levels whose two children sit in one wave (leaf = lane / G
// within a wave of 64 lanes: 2 * half * G divides 64) pass the right child's
// record with cross-lane moves instead of LDS and a block barrier.  Measured,
// this pays for the small tridiagonal records and the one-wave trees (G = 1),
// and in the long-system and uneven-batch tile kernels; in the single-launch
// split kernel a pentadiagonal record (20 doubles, 40 moves per level) costs
// as much as the LDS round trip it replaces, so that one keeps LDS.
template <int G>
__device__ constexpr bool in_wave(int half) {
  return 2 * half * G <= 64 && 64 % (2 * half * G) == 0;
}
template <typename R>
__device__ inline R shfl_down_rec(const R& r, int delta) {
  R out;
  const double* src = reinterpret_cast<const double*>(&r);
  double* dst = reinterpret_cast<double*>(&out);
#pragma unroll
  for (int q = 0; q < (int)(sizeof(R) / sizeof(double)); ++q) dst[q] = __shfl_down(src[q], delta, 64);
  return out;
}

template <int NB, int NL, int G, bool LANES = (NB == 1 || G == 1)>
__device__ inline void tree_up(Map<NB>& mp, int leaf, int g, double* s_node,
                               int* s_bad, int64_t leaf_rows, int64_t row0, int64_t n) {
  constexpr int RS = kRecSz<NB>;
  constexpr int L = __builtin_ctz(NL);
  const bool active = leaf < NL;
  int node_off = 0;
#pragma unroll
  for (int lvl = 1; lvl <= L; ++lvl) {
    const int stride = 1 << lvl, half = stride >> 1;
    const int k = leaf >> lvl;
    double* slot = s_node + ((node_off + k) * G + g) * RS;
    Map<NB> rb;
    if (LANES && in_wave<G>(half)) {  // uniform: every lane takes part in the moves
      rb = shfl_down_rec(mp, half * G);
    } else {
      if (active && (leaf & (stride - 1)) == half) store_rec(mp, slot);
      __syncthreads();
      if (active && (leaf & (stride - 1)) == 0) load_rec(rb, slot);
    }
    if (active && (leaf & (stride - 1)) == 0) {
      Node<NB> nd;
      if (!merge<NB>(mp, rb, mp, nd)) {
        const int64_t row = row0 + (int64_t)(leaf + half) * leaf_rows - NB;
        if (row < n) atomicMin(&s_bad[g], (int)(row + 1));
      }
      store_rec(nd, slot);  // read back by this lane on the way down
    }
    node_off += NL >> lvl;
  }
}

// Walk back down: on entry the lanes with leaf == 0 hold the outer pairs of
// the whole range; on exit every lane with leaf < NL holds its leaf's pairs.
// The caller puts a barrier between tree_up and tree_down.
template <int NB, int NL, int G, bool LANES = (NB == 1 || G == 1)>
__device__ inline void tree_down(double (&xl)[NB], double (&xr)[NB], int leaf, int g,
                                 double* s_node) {
  constexpr int RS = kRecSz<NB>;
  constexpr int L = __builtin_ctz(NL);
  const bool active = leaf < NL;
  int node_off = NL - 1;
#pragma unroll
  for (int lvl = L; lvl >= 1; --lvl) {
    const int stride = 1 << lvl, half = stride >> 1;
    const int k = leaf >> lvl;
    node_off -= NL >> lvl;
    double* slot = s_node + ((node_off + k) * G + g) * RS;
    double ba[NB], xr0[NB];  // the right part's pairs: x_L = B_A, x_R unchanged
#pragma unroll
    for (int q = 0; q < NB; ++q) ba[q] = xr0[q] = 0.0;
    if (active && (leaf & (stride - 1)) == 0) {
      Node<NB> nd;
      load_rec(nd, slot);
      double tb[NB], t1[NB], t2[NB];
      mv<NB>(nd.G1, xl, t1);
      mv<NB>(nd.G2, xr, t2);
#pragma unroll
      for (int q = 0; q < NB; ++q) ba[q] = nd.g0[q] + t1[q] + t2[q];
      mv<NB>(nd.H1, xl, t1);
      mv<NB>(nd.H2, xr, t2);
#pragma unroll
      for (int q = 0; q < NB; ++q) tb[q] = nd.h0[q] + t1[q] + t2[q];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        xr0[q] = xr[q];
        xr[q] = tb[q];  // left part: x_R = T_B
      }
    }
    if (LANES && in_wave<G>(half)) {  // uniform: every lane takes part in the moves
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const double bl = __shfl_up(ba[q], half * G, 64);
        const double br = __shfl_up(xr0[q], half * G, 64);
        if (active && (leaf & (stride - 1)) == half) {
          xl[q] = bl;
          xr[q] = br;
        }
      }
    } else {
      if (active && (leaf & (stride - 1)) == 0) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          slot[q] = ba[q];
          slot[NB + q] = xr0[q];
        }
      }
      __syncthreads();
      if (active && (leaf & (stride - 1)) == half) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          xl[q] = slot[q];
          xr[q] = slot[NB + q];
        }
      }
    }
  }
}

__device__ inline unsigned ld_counter(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Device-coherent (write-through / cache-bypassing) accesses for data that
// blocks on other XCDs read.
__device__ inline void st_coherent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double ld_coherent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
constexpr int kWaitVmem = 0x0F70;  // s_waitcnt vmcnt(0): this wave's memory ops done

constexpr int kBadNone = INT_MAX;
constexpr int kBadList = -3;

// MNPDM's outer diagonals as a list per system: entry k of system s is row
// row[k*ld + s] (-1 = unused) with e = e[k*ld + s], b = b[k*ld + s].
struct Outer {
  int32_t kmax;
  const int32_t* row;
  const double* e;
  const double* b;
};
constexpr int kTimeout = -4;
__device__ inline void st_coherent_i32(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads the M rows of a chunk (first row r0) of system s into registers:
// identity rows past n, zero couplings outside the matrix.  Byte offsets fit
// in 32 bits (checked on the host), so every load is an SGPR base plus one
// per-row VGPR offset shared by the six arrays.
template <int KIND, int M, typename TIO, bool OUTER = true>
__device__ inline void load_chunk(int64_t n, int64_t ld, int64_t s, bool live, int64_t r0,
                                  int64_t row_base,
                                  const TIO* __restrict__ E, const TIO* __restrict__ C,
                                  const TIO* __restrict__ D, const TIO* __restrict__ A,
                                  const TIO* __restrict__ B, const TIO* __restrict__ Y,
                                  double (&e)[M], double (&c)[M], double (&d)[M],
                                  double (&a)[M], double (&b)[M], double (&y)[M]) {
  const uint32_t row_bytes = (uint32_t)(ld * sizeof(TIO));
  const uint32_t off0 = (uint32_t)((r0 * ld + s) * (int64_t)sizeof(TIO));
  if constexpr (sizeof(TIO) == 8) {
#pragma unroll
    for (int r = 0; r < M; ++r) {
      const int64_t i = row_base + r0 + r;  // global row
      const uint32_t o = off0 + (uint32_t)r * row_bytes;
      const bool in = live && i < n;
      d[r] = in ? ldg(D, o) : 1.0;
      y[r] = in ? ldg(Y, o) : 0.0;
      c[r] = (in && i >= 1) ? ldg(C, o) : 0.0;
      a[r] = (in && i <= n - 2) ? ldg(A, o) : 0.0;
      if (KIND == 5 && OUTER) {
        e[r] = (in && i >= 2) ? ldg(E, o) : 0.0;
        b[r] = (in && i <= n - 3) ? ldg(B, o) : 0.0;
      } else {
        e[r] = 0.0;
        b[r] = 0.0;
      }
    }
  } else {
    // FP32 storage: unconditional loads (slots outside the matrix read the
    // array's first element instead, and are replaced afterwards), all
    // issued before the first widening to FP64 waits for its operand.
    // Conditional loads would each sit in a branch with their widening, and
    // the chunk's loads would then complete one at a time.
    TIO re[M], rc[M], rd[M], ra[M], rb[M], ry[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      const int64_t i = row_base + r0 + r;
      const uint32_t o = off0 + (uint32_t)r * row_bytes;
      const bool in = live && i < n;
      rd[r] = ldg(D, in ? o : 0u);
      ry[r] = ldg(Y, in ? o : 0u);
      rc[r] = ldg(C, (in && i >= 1) ? o : 0u);
      ra[r] = ldg(A, (in && i <= n - 2) ? o : 0u);
      if (KIND == 5) {
        re[r] = ldg(E, (in && i >= 2) ? o : 0u);
        rb[r] = ldg(B, (in && i <= n - 3) ? o : 0u);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < M; ++r) {
      const int64_t i = row_base + r0 + r;
      const bool in = live && i < n;
      d[r] = in ? (double)rd[r] : 1.0;
      y[r] = in ? (double)ry[r] : 0.0;
      c[r] = (in && i >= 1) ? (double)rc[r] : 0.0;
      a[r] = (in && i <= n - 2) ? (double)ra[r] : 0.0;
      e[r] = (KIND == 5 && in && i >= 2) ? (double)re[r] : 0.0;
      b[r] = (KIND == 5 && in && i <= n - 3) ? (double)rb[r] : 0.0;
    }
  }
}

// Rows assembled from the sweep input v instead of loaded: one
// implicit sweep (I - tau L(k(v))) w = v of u_t = (k(u) u_x)_x, k = 1 + u^2,
// with r = tau / h^2 and k_{i+1/2} = (k(v_i) + k(v_{i+1})) / 2:
//   c_i = -r k_{i-1/2},  a_i = -r k_{i+1/2},  d_i = 1 + r (k_{i-1/2} + k_{i+1/2}),
//   rhs_i = v_i  (interior rows),
// and zero-flux boundary rows with rhs 0: first order (KIND 3) [1, -1] and
// [-1, 1]; second order (KIND 5) [-3, 4, -1] and [1, -4, 3].  Every product
// and sum is rounded on its own in this order, so the coefficients are those
// of the host generator of the same sweep to the last bit.
// Row i (0 <= i < n) of that sweep from vm = v_{i-1}, v0 = v_i, vp = v_{i+1}
// (values outside the matrix are not used).
template <int KIND>
__device__ inline void assemble_row(int64_t i, int64_t n, double vm, double v0, double vp,
                                    double r, double& e, double& c, double& d, double& a,
                                    double& b, double& y) {
#pragma clang fp contract(off)
  e = c = a = b = y = 0.0;
  d = 1.0;
  if (i == 0) {
    if (KIND == 5) {
      d = -3.0;
      a = 4.0;
      b = -1.0;
    } else {
      d = 1.0;
      a = -1.0;
    }
  } else if (i == n - 1) {
    if (KIND == 5) {
      e = 1.0;
      c = -4.0;
      d = 3.0;
    } else {
      c = -1.0;
      d = 1.0;
    }
  } else {
    const double km = 1.0 + vm * vm;
    const double k0 = 1.0 + v0 * v0;
    const double kp = 1.0 + vp * vp;
    const double hl = 0.5 * (km + k0);
    const double hr = 0.5 * (k0 + kp);
    c = -r * hl;
    a = -r * hr;
    d = 1.0 + r * (hl + hr);
    y = v0;
  }
}

// The rows of a chunk assembled from v: reads v at rows r0 - 1 .. r0 + M
// only, 8 bytes per row instead of 48.  Identity rows past n.
template <int KIND, int M>
__device__ inline void assemble_chunk(int64_t n, int64_t ld, int64_t s, bool live, int64_t r0,
                                      const double* __restrict__ V, double r, double (&e)[M],
                                      double (&c)[M], double (&d)[M], double (&a)[M],
                                      double (&b)[M], double (&y)[M]) {
  double vv[M + 2];
#pragma unroll
  for (int q = 0; q < M + 2; ++q) {
    const int64_t i = r0 - 1 + q;
    vv[q] = (live && i >= 0 && i < n)
                ? __builtin_nontemporal_load(V + (i * ld + s))
                : 0.0;
  }
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const int64_t i = r0 + q;
    if (live && i < n) {
      assemble_row<KIND>(i, n, vv[q], vv[q + 1], vv[q + 2], r, e[q], c[q], d[q], a[q], b[q],
                         y[q]);
    } else {  // identity rows past n
      e[q] = c[q] = a[q] = b[q] = y[q] = 0.0;
      d[q] = 1.0;
    }
  }
}

// The chunk's affine map: tip rows of p, V, W.
template <int NB, int M, typename TS>
__device__ inline Map<NB> chunk_map(const TS (&p)[M], const TS (&v)[NB][M],
                                    const TS (&w)[NB][M]) {
  Map<NB> mp;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    mp.pt[q] = p[q];
    mp.pb[q] = p[M - NB + q];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      mp.Vt[q][k] = v[k][q];
      mp.Wt[q][k] = w[k][q];
      mp.Vb[q][k] = v[k][M - NB + q];
      mp.Wb[q][k] = w[k][M - NB + q];
    }
  }
  return mp;
}

template <int KIND, int M>
__device__ inline void eliminate_chunk(const double (&e)[M], const double (&c)[M],
                                       const double (&d)[M], const double (&a)[M],
                                       const double (&b)[M], const double (&y)[M],
                                       double (&p)[M], double (&v)[KIND == 5 ? 2 : 1][M],
                                       double (&w)[KIND == 5 ? 2 : 1][M], int& bad) {
  if constexpr (KIND == 5)
    chunk_pd<M>(e, c, d, a, b, y, p, v[0], v[1], w[0], w[1], bad);
  else
    chunk_td<M>(c, d, a, y, p, v[0], w[0], bad);
}

template <int NB, int M, typename TIO>
__device__ inline void write_chunk(int64_t n, int64_t ld, int64_t s, bool live, int64_t r0,
                                   int64_t row_base,
                                   const double (&p)[M], const double (&v)[NB][M],
                                   const double (&w)[NB][M], const double (&xl)[NB],
                                   const double (&xr)[NB], TIO* __restrict__ X) {
  const uint32_t row_bytes = (uint32_t)(ld * sizeof(TIO));
  const uint32_t off0 = (uint32_t)((r0 * ld + s) * (int64_t)sizeof(TIO));
#pragma unroll
  for (int r = 0; r < M; ++r) {
    const int64_t i = row_base + r0 + r;
    double xv = p[r];
#pragma unroll
    for (int k = 0; k < NB; ++k) xv = fma(-v[k][r], xl[k], fma(-w[k][r], xr[k], xv));
    if (live && i < n) stg(X, off0 + (uint32_t)r * row_bytes, xv);
  }
}

// x from the compact (FP32) chunk state, in FP32.  ACC: the store adds the
// value to what X holds (x += d of a refinement step, FP64 X).
template <int NB, int M, typename TIO, bool ACC = false>
__device__ inline void write_chunk(int64_t n, int64_t ld, int64_t s, bool live, int64_t r0,
                                   int64_t row_base,
                                   const float (&p)[M], const float (&v)[NB][M],
                                   const float (&w)[NB][M], const double (&xl)[NB],
                                   const double (&xr)[NB], TIO* __restrict__ X) {
  static_assert(!ACC || sizeof(TIO) == 8, "accumulation into FP64 x");
  const uint32_t row_bytes = (uint32_t)(ld * sizeof(TIO));
  const uint32_t off0 = (uint32_t)((r0 * ld + s) * (int64_t)sizeof(TIO));
  float fl[NB], fr[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    fl[k] = (float)xl[k];
    fr[k] = (float)xr[k];
  }
#pragma unroll
  for (int r = 0; r < M; ++r) {
    const int64_t i = row_base + r0 + r;
    float xv = p[r];
#pragma unroll
    for (int k = 0; k < NB; ++k) xv = fmaf(-v[k][r], fl[k], fmaf(-w[k][r], fr[k], xv));
    if (live && i < n) {
      TIO* dst = reinterpret_cast<TIO*>(reinterpret_cast<char*>(X) + off0 + (uint32_t)r * row_bytes);
      if constexpr (ACC)
        *dst = *dst + (double)xv;
      else
        __builtin_nontemporal_store((TIO)xv, dst);
    }
  }
}

// ---- streamed chunk: loads interleaved with the forward elimination -----
// The rows come through raw buffer loads: one 32-bit byte offset per row and
// array on a buffer resource whose range is the array, so a slot outside
// the matrix (a corner slot, a row past n, a padding system) is an offset
// past the range and reads as zero without a branch.  The loads of row
// r + D are issued at the start of row r's forward step, so the elimination
// of the rows that have arrived runs while later rows are in flight (a wave
// holds at most 63 loads: D = 10 rows of six arrays).
constexpr uint32_t kOOB = 0xFFFFFFF8u;  // beyond any array (n ld bytes < 2^32 - ld)

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <typename TIO>
__device__ inline __amdgpu_buffer_rsrc_t rsrc_of(const TIO* p, uint32_t bytes) {
  // raw buffer, byte offsets, range checked against `bytes`
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<TIO*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename TIO>
__device__ inline TIO bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(TIO) == 8)
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 2));
  else
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 2));
}

// LIST: the outer diagonals e, b are not loaded but taken from eo, bo (an
// MNPDM list scattered into registers); only c, d, a, y are streamed.
// TS: state type (double, or float for the compact state of FP32 storage).
template <int KIND, int M, int D, typename TIO, bool LIST = false, typename TS = double>
__device__ inline void stream_eliminate(int64_t n, int64_t ld, int64_t s, bool live, int64_t r0,
                                        const TIO* __restrict__ E, const TIO* __restrict__ C,
                                        const TIO* __restrict__ Dg, const TIO* __restrict__ A,
                                        const TIO* __restrict__ B, const TIO* __restrict__ Y,
                                        const double (&eo)[M], const double (&bo)[M],
                                        TS (&p)[M], TS (&v)[KIND == 5 ? 2 : 1][M],
                                        TS (&w)[KIND == 5 ? 2 : 1][M], int& bad) {
  constexpr bool OUTER = KIND == 5 && !LIST;  // e, b streamed
  const uint32_t bytes = (uint32_t)(n * ld * (int64_t)sizeof(TIO));
  const uint32_t row_bytes = (uint32_t)(ld * sizeof(TIO));
  const uint32_t off0 = (uint32_t)((r0 * ld + s) * (int64_t)sizeof(TIO));
  __amdgpu_buffer_rsrc_t rE = rsrc_of(OUTER ? E : C, bytes), rC = rsrc_of(C, bytes),
                         rD = rsrc_of(Dg, bytes), rA = rsrc_of(A, bytes),
                         rB = rsrc_of(OUTER ? B : C, bytes), rY = rsrc_of(Y, bytes);
  TIO xe[M], xc[M], xd[M], xa[M], xb[M], xy[M];
  auto issue = [&](int q) {
    const int64_t i = r0 + q;
    const uint32_t o = (live && i < n) ? off0 + (uint32_t)q * row_bytes : kOOB;
    xd[q] = bload<TIO>(rD, o);
    xy[q] = bload<TIO>(rY, o);
    xc[q] = bload<TIO>(rC, i >= 1 ? o : kOOB);
    xa[q] = bload<TIO>(rA, i <= n - 2 ? o : kOOB);
    if (OUTER) {
      xe[q] = bload<TIO>(rE, i >= 2 ? o : kOOB);
      xb[q] = bload<TIO>(rB, i <= n - 3 ? o : kOOB);
    }
  };
#pragma unroll
  for (int q = 0; q < D && q < M; ++q) issue(q);
  auto pre = [&](int r) {
    if (r + D < M) issue(r + D);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads of row r + D here
  };
  auto src = [&](int r, double& er, double& cr, double& dr, double& ar, double& br, double& yr) {
    const bool in = live && r0 + r < n;
    er = OUTER ? (double)xe[r] : (LIST ? eo[r] : 0.0);
    cr = (double)xc[r];
    dr = in ? (double)xd[r] : 1.0;  // identity rows past n
    ar = (double)xa[r];
    br = OUTER ? (double)xb[r] : (LIST ? bo[r] : 0.0);
    yr = (double)xy[r];
  };
  if constexpr (KIND == 5)
    chunk_pd_rows<M>(src, pre, p, v[0], v[1], w[0], w[1], bad);
  else
    chunk_td_rows<M>(src, pre, p, v[0], w[0], bad);
}

// The ADI sweep's rows assembled from v (assemble_row) as v arrives: all
// M + 2 values of v the chunk needs are requested at once (out-of-range rows
// read zero), and row r is assembled and eliminated once v_{r+1} is in.
template <int KIND, int M>
__device__ inline void stream_assemble(int64_t n, int64_t ld, int64_t s, bool live, int64_t r0,
                                       const double* __restrict__ V, double rcoef, double (&p)[M],
                                       double (&v)[KIND == 5 ? 2 : 1][M],
                                       double (&w)[KIND == 5 ? 2 : 1][M], int& bad) {
  const uint32_t bytes = (uint32_t)(n * ld * 8);
  const uint32_t row_bytes = (uint32_t)(ld * 8);
  __amdgpu_buffer_rsrc_t rV = rsrc_of(V, bytes);
  double vv[M + 2];  // v at rows r0 - 1 .. r0 + M
#pragma unroll
  for (int q = 0; q < M + 2; ++q) {
    const int64_t i = r0 - 1 + q;
    vv[q] = bload<double>(rV, (live && i >= 0 && i < n)
                                  ? (uint32_t)((i * ld + s) * 8)
                                  : kOOB);
  }
  (void)row_bytes;
  __builtin_amdgcn_sched_barrier(0);
  auto src = [&](int r, double& er, double& cr, double& dr, double& ar, double& br, double& yr) {
    const int64_t i = r0 + r;
    if (live && i < n) {
      assemble_row<KIND>(i, n, vv[r], vv[r + 1], vv[r + 2], rcoef, er, cr, dr, ar, br, yr);
    } else {  // identity rows past n
      er = cr = ar = br = yr = 0.0;
      dr = 1.0;
    }
  };
  if constexpr (KIND == 5)
    chunk_pd_rows<M>(src, [](int) {}, p, v[0], v[1], w[0], w[1], bad);
  else
    chunk_td_rows<M>(src, [](int) {}, p, v[0], w[0], bad);
}

}  // namespace split
}  // namespace bs
