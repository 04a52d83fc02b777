// sip_lane.hip -- the Stone method (SIP) over band ILU(0) factors, with exact
// triangular solves or Hotelling-Bodewig approximate inverses (Veneva &
// Ayriyan, arXiv:1804.09666, Sec. 2 Algorithm 1, Remark of Sec. 2, Appendix).
//
// One lane per system, one persistent launch: every lane iterates its own
// system to its own tolerance; nothing returns to the host between steps.
// Each step is two streaming passes over the rows of the system:
//   forward  -- residual r = b - A x (and its inf-norm), then w = X_L r
//               (or the exact forward substitution, or, for Algorithm 1 as
//               written, the forward solve of L w = K x + b);
//   backward -- x += X_U w (or the exact back substitution).
// The convergence test on ||r||_inf is made between the two passes.
//
// Hotelling-Bodewig without forming X: with X_0 = diag(T)^{-1} and
// G = I - X_0 T, s HB steps give X_s = sum_{m < 2^s} G^m X_0, i.e. M = 2^s
// Jacobi sweeps y_t = X_0 (v - (T - D) y_{t-1}).  Because T is triangular with
// bandwidth 2, sweep t at row i needs sweep t-1 only at rows i-1, i-2 (L) or
// i+1, i+2 (U); the M sweeps therefore run as an M-stage pipeline inside the
// single streaming pass, with 2M values of state per lane in registers.
#include "bs_internal.h"
#include "lane_stream.h"

#pragma clang fp contract(off)

namespace bs {
namespace {

constexpr int kSipBlock = 64;

__device__ inline bool bad_pivot(double m) { return !(m != 0.0) || !isfinite(m); }

template <int MMAX>
__global__ __launch_bounds__(kSipBlock) void sip_lane_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ E,
    const double* __restrict__ C, const double* __restrict__ D,
    const double* __restrict__ A, const double* __restrict__ B,
    const double* __restrict__ F, int64_t fld, const double* __restrict__ Y,
    double* __restrict__ X, double tol, int32_t max_iter, int ML, int MU,
    int32_t* __restrict__ iters, double* __restrict__ relres,
    int32_t* __restrict__ info, double* __restrict__ V, int64_t lw) {
  const int64_t s = (int64_t)blockIdx.x * kSipBlock + threadIdx.x;
  if (s >= batch) return;
  const int64_t plane = n * fld;
  const double* L2 = F;
  const double* L1 = F + plane;
  const double* U0 = F + 2 * plane;
  const double* U1 = F + 3 * plane;
  const bool exactL = ML <= 0, exactU = MU <= 0;
  const bool literal = exactL && exactU;

  // ||b||_inf and the usability of the ILU(0) pivots are gathered in the first
  // forward pass (it reads y and u0 anyway): a zero right-hand side has the
  // solution x = 0 and needs no step; a zero or non-finite u0 would make every
  // step undefined.  That pass's other results are then dropped.
  double bnorm = 0.0;
  int64_t bad = -1;
  bool first = true;

  double relres0 = -1.0, rr = 0.0;
  int32_t k = 0, status = -1;
  for (;;) {
    // ---------------- forward pass: residual, then L-side operator -------
    double rmax = 0.0;
    bool nonfinite = false;
    double xm2 = 0.0, xm1 = 0.0;
    double x0v = X[s];
    double xp1 = (n > 1) ? X[ld + s] : 0.0;
    double pl1[MMAX], pl2[MMAX];  // HB-L stages at rows i-1, i-2
#pragma unroll
    for (int t = 0; t < MMAX; ++t) pl1[t] = pl2[t] = 0.0;
    double wm1 = 0.0, wm2 = 0.0;  // exact L solve: w_{i-1}, w_{i-2}
    // Algorithm 1 as written: K = LU - A on the fly from factor rows i-1, i-2
    double u0m1 = 0, u0m2 = 0, u1m1 = 0, u1m2 = 0, u2m1 = 0, u2m2 = 0;
    constexpr int PFF = MMAX >= 64 ? 1 : 5;  // 11 loads + 1 store per row: 60 memory operations in flight; registers at 64 stages
    double rx2[PFF], re[PFF], rc[PFF], rd[PFF], ra[PFF], rb[PFF], ry[PFF], rl2[PFF], rl1[PFF],
        ru0[PFF], ru1[PFF];
    auto fetch = [&](int q, int64_t i) {
      const int64_t o = i * ld + s;
      const int64_t fo = i * fld + s;
      rx2[q] = X[(i + 2 < n ? i + 2 : i) * ld + s];
      re[q] = E[o];
      rc[q] = C[o];
      rd[q] = D[o];
      ra[q] = A[o];
      rb[q] = B[o];
      ry[q] = Y[o];
      rl2[q] = L2[fo];
      rl1[q] = L1[fo];
      ru0[q] = U0[fo];
      ru1[q] = U1[fo];
    };
    auto use = [&](int q, int64_t i) {
      // corner slots of A and the factors outside the band are never used
      const double xp2 = (i + 2 < n) ? rx2[q] : 0.0;
      const double ei = (i >= 2) ? re[q] : 0.0;
      const double ci = (i >= 1) ? rc[q] : 0.0;
      const double di = rd[q];
      const double ai = (i + 1 < n) ? ra[q] : 0.0;
      const double bi = (i + 2 < n) ? rb[q] : 0.0;
      double ax = di * x0v;
      if (i >= 2) ax = ax + ei * xm2;
      if (i >= 1) ax = ax + ci * xm1;
      if (i + 1 < n) ax = ax + ai * xp1;
      if (i + 2 < n) ax = ax + bi * xp2;
      const double yi = ry[q];
      if (first) {
        bnorm = fmax(bnorm, fabs(yi));
        if (bad < 0 && bad_pivot(ru0[q])) bad = i;
      }
      const double r = yi - ax;
      const double ar = fabs(r);
      if (!isfinite(ar)) nonfinite = true;
      rmax = fmax(rmax, ar);
      const double l2 = (i >= 2) ? rl2[q] : 0.0;
      const double l1 = (i >= 1) ? rl1[q] : 0.0;
      double wi;
      if (literal) {
        const double u0 = ru0[q];
        const double u1 = (i + 1 < n) ? ru1[q] : 0.0;
        // v = K x + b with K = LU - A, then w = L^{-1} v
        double kx = ((u0 + (i >= 1 ? l1 * u1m1 : 0.0) + (i >= 2 ? l2 * u2m2 : 0.0)) - di) * x0v;
        if (i >= 2) kx = kx + (l2 * u0m2 - ei) * xm2;
        if (i >= 1) kx = kx + (((i >= 2 ? l2 * u1m2 : 0.0) + l1 * u0m1) - ci) * xm1;
        if (i + 1 < n) kx = kx + ((u1 + (i >= 1 ? l1 * u2m1 : 0.0)) - ai) * xp1;
        const double v = kx + yi;
        wi = (v - l1 * wm1) - l2 * wm2;
        wm2 = wm1;
        wm1 = wi;
        u0m2 = u0m1; u0m1 = u0;
        u1m2 = u1m1; u1m1 = u1;
        u2m2 = u2m1; u2m1 = bi;
      } else if (exactL) {
        wi = (r - l1 * wm1) - l2 * wm2;
        wm2 = wm1;
        wm1 = wi;
      } else {
        // stage t: y_t[i] = r_i - l1_i y_{t-1}[i-1] - l2_i y_{t-1}[i-2]
#pragma unroll
        for (int t = MMAX - 1; t >= 1; --t) {
          if (t < ML) {
            const double nv = (r - l1 * pl1[t - 1]) - l2 * pl2[t - 1];
            pl2[t] = pl1[t];
            pl1[t] = nv;
          }
        }
        pl2[0] = pl1[0];
        pl1[0] = r;
        wi = r;
#pragma unroll
        for (int t = 1; t < MMAX; ++t)
          if (t == ML - 1) wi = pl1[t];
      }
      V[i * lw + s] = wi;
      xm2 = xm1;
      xm1 = x0v;
      x0v = xp1;
      xp1 = xp2;
    };
    stream_rows<PFF, false>(n, fetch, use);
    if (first) {
      first = false;
      if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) X[i * ld + s] = 0.0;
        iters[s] = 0;
        relres[s] = 0.0;
        info[s] = 0;
        return;
      }
      if (bad >= 0) {
        iters[s] = 0;
        relres[s] = NAN;
        info[s] = (int32_t)(bad + 1);
        return;
      }
    }
    rr = nonfinite ? NAN : rmax / bnorm;
    if (relres0 < 0.0) relres0 = rr;
    if (!isfinite(rr)) { status = -2; break; }
    if (!(rmax >= tol * bnorm)) { status = 0; break; }
    if (rr > 1e3 * fmax(1.0, relres0)) { status = -2; break; }
    if (k == max_iter) { status = -1; break; }

    // ---------------- backward pass: U-side operator, update x -----------
    double pu1[MMAX], pu2[MMAX];  // HB-U stages at rows i+1, i+2
#pragma unroll
    for (int t = 0; t < MMAX; ++t) pu1[t] = pu2[t] = 0.0;
    double qp1 = 0.0, qp2 = 0.0;  // exact U solve: q_{i+1}, q_{i+2}
    constexpr int PFB = MMAX >= 64 ? 1 : 10;  // 5 loads + 1 store per row: 60 in flight
    double bv[PFB], bu0[PFB], bu1[PFB], bu2[PFB], bx[PFB];
    auto fetchb = [&](int q, int64_t i) {
      const int64_t o = i * ld + s;
      const int64_t fo = i * fld + s;
      bv[q] = V[i * lw + s];
      bu0[q] = U0[fo];
      bu1[q] = U1[fo];
      bu2[q] = B[o];
      bx[q] = X[o];
    };
    auto useb = [&](int q, int64_t i) {
      const double v = bv[q];
      const double u0 = bu0[q];
      const double u1 = (i + 1 < n) ? bu1[q] : 0.0;
      const double u2 = (i + 2 < n) ? bu2[q] : 0.0;
      double qv;
      if (exactU) {
        qv = ((v - u1 * qp1) - u2 * qp2) / u0;
        qp2 = qp1;
        qp1 = qv;
      } else {
        // stage t: y_t[i] = (v_i - u1_i y_{t-1}[i+1] - u2_i y_{t-1}[i+2]) / u0_i
        const double inv = 1.0 / u0;
#pragma unroll
        for (int t = MMAX - 1; t >= 1; --t) {
          if (t < MU) {
            const double nv = ((v - u1 * pu1[t - 1]) - u2 * pu2[t - 1]) * inv;
            pu2[t] = pu1[t];
            pu1[t] = nv;
          }
        }
        pu2[0] = pu1[0];
        pu1[0] = v * inv;
        qv = pu1[0];
#pragma unroll
        for (int t = 1; t < MMAX; ++t)
          if (t == MU - 1) qv = pu1[t];
      }
      X[i * ld + s] = literal ? qv : bx[q] + qv;
    };
    stream_rows<PFB, true>(n, fetchb, useb);
    ++k;
  }
  iters[s] = k;
  relres[s] = rr;
  info[s] = status;
}

template <int MMAX>
void launch_mmax(int64_t n, int64_t batch, int64_t ld, Diags A,
                 const double* F, int64_t fld, const double* y, double* x, double tol,
                 int32_t max_iter, int ML, int MU, int32_t* iters,
                 double* relres, int32_t* info, double* V, hipStream_t st) {
  hipLaunchKernelGGL(sip_lane_kernel<MMAX>,
                     dim3((unsigned)((batch + kSipBlock - 1) / kSipBlock)),
                     dim3(kSipBlock), 0, st, n, batch, ld, A.e, A.c, A.d, A.a,
                     A.b, F, fld, y, x, tol, max_iter, ML, MU, iters, relres, info,
                     V, ws_ld(batch));
}

}  // namespace

// s < 0, or 2^s >= n: exact solve (M = 0).  Otherwise M = 2^s <= 64.
static int hb_stages(int32_t s, int64_t n) {
  if (s < 0) return 0;
  if (s >= 62 || (int64_t(1) << s) >= n) return 0;
  return 1 << s;
}

hipError_t launch_sip_lane(int64_t n, int64_t batch, int64_t ld, Diags A,
                           const double* factors, int64_t fld,
                           const double* y, double* x,
                           double tol, int32_t max_iter, int32_t sL,
                           int32_t sU, int32_t* iters, double* relres,
                           int32_t* info, double* v_ws, hipStream_t st) {
  const int ML = hb_stages(sL, n), MU = hb_stages(sU, n);
  const int M = ML > MU ? ML : MU;
  if (M <= 1)
    launch_mmax<1>(n, batch, ld, A, factors, fld, y, x, tol, max_iter, ML, MU, iters, relres, info, v_ws, st);
  else if (M <= 4)
    launch_mmax<4>(n, batch, ld, A, factors, fld, y, x, tol, max_iter, ML, MU, iters, relres, info, v_ws, st);
  else if (M <= 16)
    launch_mmax<16>(n, batch, ld, A, factors, fld, y, x, tol, max_iter, ML, MU, iters, relres, info, v_ws, st);
  else
    launch_mmax<64>(n, batch, ld, A, factors, fld, y, x, tol, max_iter, ML, MU, iters, relres, info, v_ws, st);
  return hipGetLastError();
}

}  // namespace bs
