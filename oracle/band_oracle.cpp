// band_oracle.cpp -- plain, slow, obviously correct FP64 CPU oracle for the
// batched band-SLAE methods of Veneva & Ayriyan, "Performance Analysis of
// Effective Methods for Solving Band Matrix SLAEs after Parabolic Nonlinear
// PDEs" (arXiv:1804.09666).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark do.  It shares no source, header, table or helper with
// the HIP path.
//
// Conventions (one system at a time, system-contiguous arrays of length n,
// 0-based rows).  Row i of a pentadiagonal (PD) system reads
//     e[i] x[i-2] + c[i] x[i-1] + d[i] x[i] + a[i] x[i+1] + b[i] x[i+2] = y[i]
// and a tridiagonal (TD) system drops e and b.  Any term whose column index
// falls outside 0..n-1 is omitted (never multiplied by zero), so the corner
// slots e[0], e[1], c[0], a[n-1], b[n-2], b[n-1] are never read.
//
// Arithmetic: IEEE binary64, round to nearest, true division, no contraction
// (built with -ffp-contract=off, no fast-math).  Expressions are evaluated
// left to right exactly as bracketed in the comments.
//
// Built twice: once with `real` = double (liboracle.so) and once with `real`
// = a counting wrapper (liboracle_count.so, -DORC_COUNT_FLOPS) so that a test
// can compare the number of floating-point operations the oracle performs with
// the complexity table of the paper (Sec. 4, table "Complexity of the
// investigated methods").

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#ifdef ORC_COUNT_FLOPS
static long long g_flops = 0;
struct real {
  double v;
  real() : v(0.0) {}
  real(double x) : v(x) {}
};
static inline real operator+(real p, real q) { ++g_flops; return real(p.v + q.v); }
static inline real operator-(real p, real q) { ++g_flops; return real(p.v - q.v); }
static inline real operator*(real p, real q) { ++g_flops; return real(p.v * q.v); }
static inline real operator/(real p, real q) { ++g_flops; return real(p.v / q.v); }
static inline real operator-(real p) { return real(-p.v); }
static inline double val(real p) { return p.v; }
#else
typedef double real;
static inline double val(double p) { return p; }
#endif

static inline bool bad_pivot(real p) {
  double v = val(p);
  return v == 0.0 || !std::isfinite(v);
}

extern "C" {

long long orc_flops_get(void) {
#ifdef ORC_COUNT_FLOPS
  return g_flops;
#else
  return -1;
#endif
}

void orc_flops_reset(void) {
#ifdef ORC_COUNT_FLOPS
  g_flops = 0;
#endif
}

// ---------------------------------------------------------------------------
// NPDM: numerical method for a pentadiagonal matrix (Sec. 1; complexity
// 19N-29 in the complexity table of Sec. 4).  LU without pivoting with
// L = (e, gamma, mu) on diagonals -2, -1, 0 and U unit upper with
// (alpha, beta) on +1, +2:
//   gamma_i = c_i - alpha_{i-2} e_i
//   mu_i    = (d_i - beta_{i-2} e_i) - alpha_{i-1} gamma_i
//   alpha_i = (a_i - beta_{i-1} gamma_i) / mu_i          (i <= n-2)
//   beta_i  = b_i / mu_i                                  (i <= n-3)
//   z_i     = ((y_i - z_{i-2} e_i) - z_{i-1} gamma_i) / mu_i
//   x_{n-1} = z_{n-1},  x_i = (z_i - alpha_i x_{i+1}) - beta_i x_{i+2}.
// Returns 0, or i+1 for the first pivot mu_i that is zero or not finite (x is
// then left unspecified).  `mu_out` (nullable) receives the pivots, whose
// product is det A.
// ---------------------------------------------------------------------------
int orc_npdm(int64_t n, const double* e, const double* c, const double* d,
             const double* a, const double* b, const double* y, double* x,
             double* mu_out) {
  std::vector<real> alpha(n), beta(n), z(n);
  for (int64_t i = 0; i < n; ++i) {
    real gamma = 0.0, mu = 0.0;
    if (i == 0) {
      mu = d[0];
    } else if (i == 1) {
      gamma = c[1];
      mu = real(d[1]) - alpha[0] * gamma;
    } else {
      gamma = real(c[i]) - alpha[i - 2] * e[i];
      mu = (real(d[i]) - beta[i - 2] * e[i]) - alpha[i - 1] * gamma;
    }
    if (mu_out) mu_out[i] = val(mu);
    if (bad_pivot(mu)) return (int)(i + 1);
    if (i <= n - 2) {
      if (i == 0)
        alpha[0] = real(a[0]) / mu;
      else
        alpha[i] = (real(a[i]) - beta[i - 1] * gamma) / mu;
    }
    if (i <= n - 3) beta[i] = real(b[i]) / mu;
    if (i == 0)
      z[0] = real(y[0]) / mu;
    else if (i == 1)
      z[1] = (real(y[1]) - z[0] * gamma) / mu;
    else
      z[i] = ((real(y[i]) - z[i - 2] * e[i]) - z[i - 1] * gamma) / mu;
  }
  std::vector<real> xs(n);
  for (int64_t i = n - 1; i >= 0; --i) {
    if (i == n - 1)
      xs[i] = z[i];
    else if (i == n - 2)
      xs[i] = z[i] - alpha[i] * xs[i + 1];
    else
      xs[i] = (z[i] - alpha[i] * xs[i + 1]) - beta[i] * xs[i + 2];
  }
  for (int64_t i = 0; i < n; ++i) x[i] = val(xs[i]);
  return 0;
}

// ---------------------------------------------------------------------------
// NTDM: numerical method for a tridiagonal matrix, i.e. the Thomas algorithm
// (Sec. 1), in division form:
//   mu_0 = d_0,  mu_i = d_i - alpha_{i-1} c_i,  alpha_i = a_i / mu_i,
//   z_i = (y_i - z_{i-1} c_i) / mu_i,  x_i = z_i - alpha_i x_{i+1}.
// Same return convention as orc_npdm.
// ---------------------------------------------------------------------------
int orc_ntdm(int64_t n, const double* c, const double* d, const double* a,
             const double* y, double* x, double* mu_out) {
  std::vector<real> alpha(n), z(n);
  for (int64_t i = 0; i < n; ++i) {
    real mu;
    if (i == 0)
      mu = d[0];
    else
      mu = real(d[i]) - alpha[i - 1] * c[i];
    if (mu_out) mu_out[i] = val(mu);
    if (bad_pivot(mu)) return (int)(i + 1);
    if (i <= n - 2) alpha[i] = real(a[i]) / mu;
    if (i == 0)
      z[0] = real(y[0]) / mu;
    else
      z[i] = (real(y[i]) - z[i - 1] * c[i]) / mu;
  }
  std::vector<real> xs(n);
  for (int64_t i = n - 1; i >= 0; --i) {
    if (i == n - 1)
      xs[i] = z[i];
    else
      xs[i] = z[i] - alpha[i] * xs[i + 1];
  }
  for (int64_t i = 0; i < n; ++i) x[i] = val(xs[i]);
  return 0;
}

// ---------------------------------------------------------------------------
// MNPDM: NPDM that takes the sparsity of the first and fifth diagonals into
// account (Sec. 1; complexity 13N+7K-14, Sec. 4).  The outer diagonals are
// given as a list of K entries (rows[k], e_at[k], b_at[k]), rows strictly
// ascending; every other e_i and b_i is zero.  Every product with an absent
// (zero) e_i or beta_i is skipped, which leaves the NPDM result unchanged bit
// for bit on finite data.  Returns 0, i+1 on a bad pivot, or -3 if the list is
// not strictly ascending or names a row outside 0..n-1.
// ---------------------------------------------------------------------------
int orc_mnpdm(int64_t n, const double* c, const double* d, const double* a,
              int64_t k, const int64_t* rows, const double* e_at,
              const double* b_at, const double* y, double* x) {
  std::vector<double> e(n, 0.0), bb(n, 0.0);
  std::vector<char> has_e(n, 0), has_b(n, 0);
  for (int64_t q = 0; q < k; ++q) {
    int64_t r = rows[q];
    if (r < 0 || r >= n || (q > 0 && r <= rows[q - 1])) return -3;
    if (r >= 2 && e_at[q] != 0.0) { e[r] = e_at[q]; has_e[r] = 1; }
    if (r <= n - 3 && b_at[q] != 0.0) { bb[r] = b_at[q]; has_b[r] = 1; }
  }
  std::vector<real> alpha(n), beta(n), z(n);
  for (int64_t i = 0; i < n; ++i) {
    real gamma = 0.0, mu = 0.0;
    if (i == 0) {
      mu = d[0];
    } else {
      gamma = c[i];
      if (has_e[i]) gamma = real(c[i]) - alpha[i - 2] * e[i];
      mu = d[i];
      if (has_e[i] && has_b[i - 2]) mu = real(d[i]) - beta[i - 2] * e[i];
      mu = mu - alpha[i - 1] * gamma;
    }
    if (bad_pivot(mu)) return (int)(i + 1);
    if (i <= n - 2) {
      if (i >= 1 && has_b[i - 1])
        alpha[i] = (real(a[i]) - beta[i - 1] * gamma) / mu;
      else
        alpha[i] = real(a[i]) / mu;
    }
    if (has_b[i]) beta[i] = real(bb[i]) / mu;
    if (i == 0)
      z[0] = real(y[0]) / mu;
    else if (has_e[i])
      z[i] = ((real(y[i]) - z[i - 2] * e[i]) - z[i - 1] * gamma) / mu;
    else
      z[i] = (real(y[i]) - z[i - 1] * gamma) / mu;
  }
  std::vector<real> xs(n);
  for (int64_t i = n - 1; i >= 0; --i) {
    if (i == n - 1)
      xs[i] = z[i];
    else if (has_b[i])
      xs[i] = (z[i] - alpha[i] * xs[i + 1]) - beta[i] * xs[i + 2];
    else
      xs[i] = z[i] - alpha[i] * xs[i + 1];
  }
  for (int64_t i = 0; i < n; ++i) x[i] = val(xs[i]);
  return 0;
}

// ---------------------------------------------------------------------------
// ILU(0) of a pentadiagonal matrix (Sec. 2): L and U keep the zero pattern of
// A, L unit lower with (l2, l1) on diagonals -2, -1, U upper with
// (u0, u1, u2) on 0, +1, +2.  Matching (LU)_ij = a_ij on the band row by row
// (Doolittle order) gives
//   l2_i = e_i / u0_{i-2}
//   l1_i = (c_i - l2_i u1_{i-2}) / u0_{i-1}
//   u0_i = (d_i - l2_i u2_{i-2}) - l1_i u1_{i-1}
//   u1_i = a_i - l1_i u2_{i-1}
//   u2_i = b_i
// (absent terms omitted; l2_0 = l2_1 = l1_0 = 0, u1_{n-1} = u2_{n-2} =
// u2_{n-1} = 0).  A band has no fill outside the band, so this is the exact
// LU of A.  Returns 0 or i+1 for the first bad u0_i.
// ---------------------------------------------------------------------------
int orc_ilu0_band(int64_t n, const double* e, const double* c, const double* d,
                  const double* a, const double* b, double* l2, double* l1,
                  double* u0, double* u1) {
  std::vector<real> L2(n), L1(n), U0(n), U1(n), U2(n);
  for (int64_t i = 0; i < n; ++i) {
    if (i >= 2) L2[i] = real(e[i]) / U0[i - 2];
    if (i == 1) L1[i] = real(c[i]) / U0[i - 1];
    if (i >= 2) L1[i] = (real(c[i]) - L2[i] * U1[i - 2]) / U0[i - 1];
    if (i == 0)
      U0[i] = d[i];
    else if (i == 1)
      U0[i] = real(d[i]) - L1[i] * U1[i - 1];
    else
      U0[i] = (real(d[i]) - L2[i] * U2[i - 2]) - L1[i] * U1[i - 1];
    if (bad_pivot(U0[i])) return (int)(i + 1);
    if (i <= n - 2) {
      if (i == 0)
        U1[i] = a[i];
      else
        U1[i] = real(a[i]) - L1[i] * U2[i - 1];
    }
    if (i <= n - 3) U2[i] = b[i];
  }
  for (int64_t i = 0; i < n; ++i) {
    l2[i] = val(L2[i]);
    l1[i] = val(L1[i]);
    u0[i] = val(U0[i]);
    u1[i] = val(U1[i]);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// ILU(0) as defined for a general sparse matrix (Sec. 2): Gaussian
// elimination in IKJ order in which only positions of the nonzero pattern are
// updated.  Dense n*n row-major storage (small n only); `pattern` holds 1 for
// positions in the pattern.  On return A holds U in its upper triangle and the
// multipliers of the unit-lower L below the diagonal.
// ---------------------------------------------------------------------------
int orc_ilu0_pattern_dense(int64_t n, double* A, const unsigned char* pattern) {
  for (int64_t i = 1; i < n; ++i) {
    for (int64_t k = 0; k < i; ++k) {
      if (!pattern[i * n + k]) continue;
      if (A[k * n + k] == 0.0) return (int)(k + 1);
      A[i * n + k] = A[i * n + k] / A[k * n + k];
      for (int64_t j = k + 1; j < n; ++j) {
        if (!pattern[i * n + j]) continue;
        A[i * n + j] = A[i * n + j] - A[i * n + k] * A[k * n + j];
      }
    }
  }
  return 0;
}

// Forward substitution with the unit lower factor, then back substitution
// with the upper factor:  z_i = (y_i - l1_i z_{i-1}) - l2_i z_{i-2},
// x_i = ((z_i - u1_i x_{i+1}) - u2_i x_{i+2}) / u0_i, with u2 = b.
static void band_lu_solve(int64_t n, const real* l2, const real* l1,
                          const real* u0, const real* u1, const real* u2,
                          const real* y, real* x) {
  std::vector<real> z(n);
  for (int64_t i = 0; i < n; ++i) {
    real t = y[i];
    if (i >= 1) t = t - l1[i] * z[i - 1];
    if (i >= 2) t = t - l2[i] * z[i - 2];
    z[i] = t;
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    real t = z[i];
    if (i + 1 < n) t = t - u1[i] * x[i + 1];
    if (i + 2 < n) t = t - u2[i] * x[i + 2];
    x[i] = t / u0[i];
  }
}

int orc_band_lu_solve(int64_t n, const double* l2, const double* l1,
                      const double* u0, const double* u1, const double* b,
                      const double* y, double* x) {
  std::vector<real> L2(l2, l2 + n), L1(l1, l1 + n), U0(u0, u0 + n),
      U1(u1, u1 + n), U2(n), Y(y, y + n), X(n);
  for (int64_t i = 0; i + 2 < n; ++i) U2[i] = b[i];
  for (int64_t i = 0; i < n; ++i)
    if (bad_pivot(U0[i])) return (int)(i + 1);
  band_lu_solve(n, L2.data(), L1.data(), U0.data(), U1.data(), U2.data(),
                Y.data(), X.data());
  for (int64_t i = 0; i < n; ++i) x[i] = val(X[i]);
  return 0;
}

// ---------------------------------------------------------------------------
// Hotelling-Bodewig iteration (Appendix, HB equation), matrix form:
//   X_{j+1} = X_j (2 I - T X_j),  X_0 = diag(T)^{-1}  (a diagonal initial
// guess, as the Remark of Sec. 2 suggests).  Dense n*n row-major, small n.
// ---------------------------------------------------------------------------
int orc_hb_matrix(int64_t n, const double* T, int s, double* X) {
  std::vector<double> Xc((size_t)(n * n), 0.0), TX((size_t)(n * n)),
      M((size_t)(n * n));
  for (int64_t i = 0; i < n; ++i) {
    if (T[i * n + i] == 0.0) return (int)(i + 1);
    Xc[i * n + i] = 1.0 / T[i * n + i];
  }
  for (int j = 0; j < s; ++j) {
    for (int64_t i = 0; i < n; ++i)  // TX = T X_j
      for (int64_t k = 0; k < n; ++k) {
        double acc = 0.0;
        for (int64_t l = 0; l < n; ++l) acc = acc + T[i * n + l] * Xc[l * n + k];
        TX[i * n + k] = acc;
      }
    for (int64_t i = 0; i < n; ++i)  // M = 2I - T X_j
      for (int64_t k = 0; k < n; ++k)
        M[i * n + k] = (i == k ? 2.0 : 0.0) - TX[i * n + k];
    std::vector<double> Xn((size_t)(n * n));
    for (int64_t i = 0; i < n; ++i)  // X_{j+1} = X_j M
      for (int64_t k = 0; k < n; ++k) {
        double acc = 0.0;
        for (int64_t l = 0; l < n; ++l) acc = acc + Xc[i * n + l] * M[l * n + k];
        Xn[i * n + k] = acc;
      }
    Xc.swap(Xn);
  }
  std::memcpy(X, Xc.data(), sizeof(double) * (size_t)(n * n));
  return 0;
}

// HB applied to a vector without forming X_s.  With G = I - X_0 T, the HB
// iterate is X_s = sum_{m < 2^s} G^m X_0, so X_s v is reached by
//   y_0 = X_0 v,  y_t = y_{t-1} + X_0 (v - T y_{t-1}),  t = 1 .. 2^s - 1.
// Lower factor: T = L (unit diagonal, X_0 = I).
static void hb_lower(int64_t n, const real* l2, const real* l1, int s,
                     const real* v, real* out) {
  std::vector<real> yo(v, v + n), yn(n);
  long long sweeps = (1LL << s) - 1;
  for (long long t = 0; t < sweeps; ++t) {
    for (int64_t i = 0; i < n; ++i) {
      real ty = yo[i];
      if (i >= 1) ty = ty + l1[i] * yo[i - 1];
      if (i >= 2) ty = ty + l2[i] * yo[i - 2];
      yn[i] = yo[i] + (v[i] - ty);
    }
    yo.swap(yn);
  }
  for (int64_t i = 0; i < n; ++i) out[i] = yo[i];
}

// Upper factor: T = U with diagonal u0, X_0 = diag(u0)^{-1}.
static void hb_upper(int64_t n, const real* u0, const real* u1, const real* u2,
                     int s, const real* v, real* out) {
  std::vector<real> yo(n), yn(n);
  for (int64_t i = 0; i < n; ++i) yo[i] = v[i] / u0[i];
  long long sweeps = (1LL << s) - 1;
  for (long long t = 0; t < sweeps; ++t) {
    for (int64_t i = 0; i < n; ++i) {
      real ty = u0[i] * yo[i];
      if (i + 1 < n) ty = ty + u1[i] * yo[i + 1];
      if (i + 2 < n) ty = ty + u2[i] * yo[i + 2];
      yn[i] = yo[i] + (v[i] - ty) / u0[i];
    }
    yo.swap(yn);
  }
  for (int64_t i = 0; i < n; ++i) out[i] = yo[i];
}

int orc_hb_lower_apply(int64_t n, const double* l2, const double* l1, int s,
                       const double* v, double* out) {
  if (s < 0 || s > 24) return -3;
  std::vector<real> L2(l2, l2 + n), L1(l1, l1 + n), V(v, v + n), O(n);
  hb_lower(n, L2.data(), L1.data(), s, V.data(), O.data());
  for (int64_t i = 0; i < n; ++i) out[i] = val(O[i]);
  return 0;
}

int orc_hb_upper_apply(int64_t n, const double* u0, const double* u1,
                       const double* b, int s, const double* v, double* out) {
  if (s < 0 || s > 24) return -3;
  std::vector<real> U0(u0, u0 + n), U1(u1, u1 + n), U2(n), V(v, v + n), O(n);
  for (int64_t i = 0; i + 2 < n; ++i) U2[i] = b[i];
  hb_upper(n, U0.data(), U1.data(), U2.data(), s, V.data(), O.data());
  for (int64_t i = 0; i < n; ++i) out[i] = val(O[i]);
  return 0;
}

// r = y - A x for the pentadiagonal A, and max |r_i|.
static real residual(int64_t n, const double* e, const double* c,
                     const double* d, const double* a, const double* b,
                     const double* y, const real* x, real* r) {
  double rmax = 0.0;
  bool nonfinite = false;
  for (int64_t i = 0; i < n; ++i) {
    real ax = real(d[i]) * x[i];
    if (i >= 2) ax = ax + real(e[i]) * x[i - 2];
    if (i >= 1) ax = ax + real(c[i]) * x[i - 1];
    if (i + 1 < n) ax = ax + real(a[i]) * x[i + 1];
    if (i + 2 < n) ax = ax + real(b[i]) * x[i + 2];
    r[i] = real(y[i]) - ax;
    double m = std::fabs(val(r[i]));
    if (!std::isfinite(m)) nonfinite = true;
    if (m > rmax) rmax = m;
  }
  return nonfinite ? real(NAN) : real(rmax);
}

// ---------------------------------------------------------------------------
// SIP / Stone method (Sec. 2, Algorithm 1) on ILU(0) factors.
//
// With s_L < 0 and s_U < 0 this is Algorithm 1 as written:
//   K = LU - A;  repeat { v = K x + b;  solve L w = v;  solve U x = w;
//                         r = b - A x;  k++ }  while ||r||_inf >= tolerance.
// Otherwise the Remark of Sec. 2 replaces the triangular solves by the
// Hotelling-Bodewig approximations X_L ~ L^{-1}, X_U ~ U^{-1} with s_L, s_U
// HB steps (a negative s keeps the exact solve for that factor).  The update
// is then applied in defect form, x <- x + X_U X_L (b - A x), which equals the
// form above when the X are exact and keeps b = A x as its fixed point when
// they are not.
//
// Stopping: converged when ||b - A x||_inf < tol * ||b||_inf (relative form of
// the paper's absolute errorMargin test).  k counts loop bodies; the test is
// made before the first body.  b = 0 gives x = 0, k = 0.
// Returns 0 (converged), -1 (max_iter reached), -2 (diverged: residual not
// finite or relres > 1e3 * max(1, relres_0)), i+1 (bad ILU(0) pivot),
// -3 (bad argument).  `x` carries x0 in and the final iterate out.
// ---------------------------------------------------------------------------
int orc_sip(int64_t n, const double* e, const double* c, const double* d,
            const double* a, const double* b, const double* y,
            const double* l2_in, const double* l1_in, const double* u0_in,
            const double* u1_in, double tol, int max_iter, int s_L, int s_U,
            double* x, int* iters, double* relres) {
  if (n < 1 || !(tol > 0.0) || max_iter < 0 || s_L > 24 || s_U > 24) return -3;
  std::vector<double> l2(n), l1(n), u0(n), u1(n);
  if (l2_in && l1_in && u0_in && u1_in) {
    std::memcpy(l2.data(), l2_in, sizeof(double) * n);
    std::memcpy(l1.data(), l1_in, sizeof(double) * n);
    std::memcpy(u0.data(), u0_in, sizeof(double) * n);
    std::memcpy(u1.data(), u1_in, sizeof(double) * n);
  } else {
    int f = orc_ilu0_band(n, e, c, d, a, b, l2.data(), l1.data(), u0.data(),
                          u1.data());
    if (f != 0) return f;
  }
  std::vector<real> L2(l2.begin(), l2.end()), L1(l1.begin(), l1.end()),
      U0(u0.begin(), u0.end()), U1(u1.begin(), u1.end()), U2(n);
  for (int64_t i = 0; i + 2 < n; ++i) U2[i] = b[i];

  double bnorm = 0.0;
  for (int64_t i = 0; i < n; ++i) bnorm = std::fmax(bnorm, std::fabs(y[i]));
  if (bnorm == 0.0) {
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    *iters = 0;
    *relres = 0.0;
    return 0;
  }

  const bool literal = (s_L < 0 && s_U < 0);
  // K = LU - A on the five diagonals (Algorithm 1): (LU)_{i,i-2} = l2_i u0_{i-2},
  // (LU)_{i,i-1} = l2_i u1_{i-2} + l1_i u0_{i-1}, (LU)_{ii} = l2_i u2_{i-2} +
  // l1_i u1_{i-1} + u0_i, (LU)_{i,i+1} = l1_i u2_{i-1} + u1_i, (LU)_{i,i+2} = u2_i.
  std::vector<real> Km2(n), Km1(n), K0(n), Kp1(n), Kp2(n);
  if (literal) {
    for (int64_t i = 0; i < n; ++i) {
      if (i >= 2) Km2[i] = L2[i] * U0[i - 2] - e[i];
      if (i >= 1) {
        real t = L1[i] * U0[i - 1];
        if (i >= 2) t = L2[i] * U1[i - 2] + t;
        Km1[i] = t - c[i];
      }
      real t0 = U0[i];
      if (i >= 1) t0 = L1[i] * U1[i - 1] + t0;
      if (i >= 2) t0 = L2[i] * U2[i - 2] + t0;
      K0[i] = t0 - d[i];
      if (i + 1 < n) {
        real t = U1[i];
        if (i >= 1) t = L1[i] * U2[i - 1] + t;
        Kp1[i] = t - a[i];
      }
      if (i + 2 < n) Kp2[i] = U2[i] - b[i];
    }
  }

  std::vector<real> X(x, x + n), R(n), V(n), W(n);
  real rn = residual(n, e, c, d, a, b, y, X.data(), R.data());
  const double relres0 = val(rn) / bnorm;
  int k = 0, status = -1;
  for (;;) {
    double rr = val(rn) / bnorm;
    if (!std::isfinite(rr)) { status = -2; break; }
    if (!(val(rn) >= tol * bnorm)) { status = 0; break; }
    if (rr > 1e3 * std::fmax(1.0, relres0)) { status = -2; break; }
    if (k == max_iter) { status = -1; break; }
    if (literal) {
      for (int64_t i = 0; i < n; ++i) {  // v = K x + b
        real t = K0[i] * X[i];
        if (i >= 2) t = t + Km2[i] * X[i - 2];
        if (i >= 1) t = t + Km1[i] * X[i - 1];
        if (i + 1 < n) t = t + Kp1[i] * X[i + 1];
        if (i + 2 < n) t = t + Kp2[i] * X[i + 2];
        V[i] = t + y[i];
      }
      band_lu_solve(n, L2.data(), L1.data(), U0.data(), U1.data(), U2.data(),
                    V.data(), X.data());
    } else {
      if (s_L < 0) {  // exact forward substitution with L
        for (int64_t i = 0; i < n; ++i) {
          real t = R[i];
          if (i >= 1) t = t - L1[i] * V[i - 1];
          if (i >= 2) t = t - L2[i] * V[i - 2];
          V[i] = t;
        }
      } else {
        hb_lower(n, L2.data(), L1.data(), s_L, R.data(), V.data());
      }
      if (s_U < 0) {  // exact back substitution with U
        for (int64_t i = n - 1; i >= 0; --i) {
          real t = V[i];
          if (i + 1 < n) t = t - U1[i] * W[i + 1];
          if (i + 2 < n) t = t - U2[i] * W[i + 2];
          W[i] = t / U0[i];
        }
      } else {
        hb_upper(n, U0.data(), U1.data(), U2.data(), s_U, V.data(), W.data());
      }
      for (int64_t i = 0; i < n; ++i) X[i] = X[i] + W[i];
    }
    rn = residual(n, e, c, d, a, b, y, X.data(), R.data());
    ++k;
  }
  for (int64_t i = 0; i < n; ++i) x[i] = val(X[i]);
  *iters = k;
  *relres = val(rn) / bnorm;
  return status;
}

// Dense Gaussian elimination (row-major, A and y overwritten), without
// (pivot = 0) or with (pivot = 1) partial pivoting.  Reference for tiny n.
int orc_dense_solve(int64_t n, double* A, double* y, double* x, int pivot) {
  for (int64_t k = 0; k < n; ++k) {
    if (pivot) {
      int64_t p = k;
      for (int64_t i = k + 1; i < n; ++i)
        if (std::fabs(A[i * n + k]) > std::fabs(A[p * n + k])) p = i;
      if (p != k) {
        for (int64_t j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
        std::swap(y[k], y[p]);
      }
    }
    if (A[k * n + k] == 0.0) return (int)(k + 1);
    for (int64_t i = k + 1; i < n; ++i) {
      double m = A[i * n + k] / A[k * n + k];
      for (int64_t j = k; j < n; ++j) A[i * n + j] = A[i * n + j] - m * A[k * n + j];
      y[i] = y[i] - m * y[k];
    }
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double t = y[i];
    for (int64_t j = i + 1; j < n; ++j) t = t - A[i * n + j] * x[j];
    x[i] = t / A[i * n + i];
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Batch drivers: `batch` independent systems, system-contiguous ([batch][n]),
// spread over `nthreads` OpenMP threads (0: the OpenMP default).  They only
// loop over the per-system routines above.
// ---------------------------------------------------------------------------
#ifdef _OPENMP
#include <omp.h>
#define ORC_THREADS(nt) num_threads((nt) > 0 ? (nt) : omp_get_max_threads())
#else
#define ORC_THREADS(nt)
#endif
#define ORC_UNUSED(v) (void)(v)

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_npdm_batch(int64_t n, int64_t batch, const double* e, const double* c,
                    const double* d, const double* a, const double* b,
                    const double* y, double* x, int32_t* info, int nthreads) {
  ORC_UNUSED(nthreads);
#pragma omp parallel for schedule(static) ORC_THREADS(nthreads)
  for (int64_t s = 0; s < batch; ++s)
    info[s] = orc_npdm(n, e + s * n, c + s * n, d + s * n, a + s * n,
                       b + s * n, y + s * n, x + s * n, nullptr);
}

void orc_ntdm_batch(int64_t n, int64_t batch, const double* c, const double* d,
                    const double* a, const double* y, double* x, int32_t* info,
                    int nthreads) {
  ORC_UNUSED(nthreads);
#pragma omp parallel for schedule(static) ORC_THREADS(nthreads)
  for (int64_t s = 0; s < batch; ++s)
    info[s] = orc_ntdm(n, c + s * n, d + s * n, a + s * n, y + s * n,
                       x + s * n, nullptr);
}

void orc_ilu0_band_batch(int64_t n, int64_t batch, const double* e,
                         const double* c, const double* d, const double* a,
                         const double* b, double* l2, double* l1, double* u0,
                         double* u1, int32_t* info, int nthreads) {
  ORC_UNUSED(nthreads);
#pragma omp parallel for schedule(static) ORC_THREADS(nthreads)
  for (int64_t s = 0; s < batch; ++s)
    info[s] = orc_ilu0_band(n, e + s * n, c + s * n, d + s * n, a + s * n,
                            b + s * n, l2 + s * n, l1 + s * n, u0 + s * n,
                            u1 + s * n);
}

void orc_sip_batch(int64_t n, int64_t batch, const double* e, const double* c,
                   const double* d, const double* a, const double* b,
                   const double* y, double tol, int max_iter, int s_L, int s_U,
                   double* x, int32_t* iters, double* relres, int32_t* status,
                   int nthreads) {
  ORC_UNUSED(nthreads);
#pragma omp parallel for schedule(dynamic) ORC_THREADS(nthreads)
  for (int64_t s = 0; s < batch; ++s) {
    int it = 0;
    double rr = 0.0;
    status[s] = orc_sip(n, e + s * n, c + s * n, d + s * n, a + s * n,
                        b + s * n, y + s * n, nullptr, nullptr, nullptr,
                        nullptr, tol, max_iter, s_L, s_U, x + s * n, &it, &rr);
    iters[s] = it;
    relres[s] = rr;
  }
}

}  // extern "C"
