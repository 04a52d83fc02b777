// sip_exact.hip -- the Stone method (SIP) as Algorithm 1 is printed (Veneva
// & Ayriyan, arXiv:1804.09666, Sec. 2): K = LU - A, then repeat
//   v = K x + b;  solve L w = v;  solve U x = w;  k++
// while ||b - A x||_inf >= tol ||b||_inf, with the rows of every system
// split over many lanes.
//
// Passes (rows of every system split over lanes; 64 systems x 4 segments
// of kRB rows per block):
//   first pass   -- every row's residual r_i = b_i - (A x0)_i, ||b||_inf,
//                   the ILU(0) pivot check and v_i = (K x0)_i + b_i (K from
//                   the factor rows i, i-1, i-2 and A's row i);
//   residual     -- after step k, r = b - A x_k only;
//   K x + b      -- after a failed test at k, v for the systems still
//                   stepping;
//   substitution -- the split L- and U-solves of direct_lane.hip on v, only
//                   for the systems still stepping; bitwise the sequential
//                   sweeps.
// The first and residual passes reduce max |r_i| per system, and their last
// block to finish applies Algorithm 1's test to every system.  (With the
// band's exact LU a system stops after one step, so the pass after it skips
// the factor reads and the v store that a step would need.)
// Every expression is the one-lane kernel's (sip_lane.hip), in its order, so
// iterates, step counts, residuals and statuses are that kernel's to the last
// bit.  max_iter steps are enqueued; once no system steps, a device flag
// makes the remaining launches return at once.
#include <climits>

#include "bs_internal.h"
#include "lane_stream.h"

#pragma clang fp contract(off)

namespace bs {
namespace {

constexpr int kRB = 32;  // rows per thread in the rv pass

constexpr int kFirst = 0, kResid = 1, kKxb = 2;  // pass kinds

struct State {
  int32_t* active;           // 1 while the system still steps
  int32_t* zero;             // 1: the answer is x = 0 (b = 0)
  int32_t* any_zero;         // some system has b = 0
  unsigned long long* rmax;  // max |r_i| of the pass in flight (bits; NaN if any is not finite)
  unsigned long long* bnorm; // ||b||_inf (bits)
  int32_t* badrow;           // first row with a bad u0 (INT_MAX: none)
  double* relres0;
  int32_t* done;
  unsigned* arrive;
};

__device__ inline bool bad_pivot(double m) { return !(m != 0.0) || !isfinite(m); }

__device__ inline double take(unsigned long long* p) {
  return __longlong_as_double((long long)__hip_atomic_exchange(p, 0ull, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT));
}

__global__ void sx_init_kernel(int64_t batch, State st) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < batch;
       s += (int64_t)gridDim.x * blockDim.x) {
    st.active[s] = 0;
    st.zero[s] = 0;
    st.rmax[s] = 0ull;
    st.bnorm[s] = 0ull;
    st.badrow[s] = INT_MAX;
    st.relres0[s] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *st.done = 0;
    *st.arrive = 0u;
    *st.any_zero = 0;
  }
}

// Block: 64 consecutive systems x 4 segments of kRB rows (one wave each).
template <int MODE>
__global__ __launch_bounds__(256) void sx_rv_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ E,
    const double* __restrict__ C, const double* __restrict__ D, const double* __restrict__ A,
    const double* __restrict__ B, const double* __restrict__ F, int64_t fld,
    const double* __restrict__ Y, const double* __restrict__ X, double* __restrict__ V,
    int64_t lw, State st, int32_t k, int32_t max_iter, double tol, int32_t* __restrict__ iters,
    double* __restrict__ relres, int32_t* __restrict__ info) {
  constexpr bool FIRST = MODE == kFirst;
  constexpr bool RES = MODE != kKxb;  // residual and test
  constexpr bool KXB = MODE != kResid;  // v = K x + b
  if (*st.done) return;
  __shared__ unsigned long long s_m[4][64], s_b[4][64];
  __shared__ int s_bad[4][64];
  __shared__ int s_last, s_any;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int64_t s = (int64_t)blockIdx.x * 64 + lane;
  const int64_t lo = ((int64_t)blockIdx.y * 4 + wv) * kRB;
  const int64_t hi = lo + kRB < n ? lo + kRB : n;
  const bool live = s < batch && lo < n && (FIRST || st.active[s] != 0);
  const int64_t plane = n * fld;
  const double* L2 = F;
  const double* L1 = F + plane;
  const double* U0 = F + 2 * plane;
  const double* U1 = F + 3 * plane;
  double rmax = 0.0, bmax = 0.0;
  bool nonfinite = false;
  int bad = INT_MAX;
  if (live) {
    // x at rows lo-2 .. lo+1 and the factor state of rows lo-1, lo-2
    double xm2 = lo >= 2 ? X[(lo - 2) * ld + s] : 0.0;
    double xm1 = lo >= 1 ? X[(lo - 1) * ld + s] : 0.0;
    double x0v = X[lo * ld + s];
    double xp1 = lo + 1 < n ? X[(lo + 1) * ld + s] : 0.0;
    double u0m1 = 0, u0m2 = 0, u1m1 = 0, u1m2 = 0, u2m1 = 0, u2m2 = 0;
    if (KXB && lo >= 1) {
      u0m1 = U0[(lo - 1) * fld + s];
      u1m1 = U1[(lo - 1) * fld + s];        // row lo - 1 < n - 1
      u2m1 = lo + 1 < n ? B[(lo - 1) * ld + s] : 0.0;
    }
    if (KXB && lo >= 2) {
      u0m2 = U0[(lo - 2) * fld + s];
      u1m2 = U1[(lo - 2) * fld + s];
      u2m2 = B[(lo - 2) * ld + s];          // row lo - 2 < n - 2
    }
    constexpr int PF = 5;  // 11 loads + 1 store per row
    double rx2[PF], re[PF], rc[PF], rd[PF], ra[PF], rb[PF], ry[PF], rl2[PF], rl1[PF], ru0[PF],
        ru1[PF];
    auto fetch = [&](int q, int64_t kk) {
      const int64_t i = lo + kk;
      const int64_t o = i * ld + s;
      const int64_t fo = i * fld + s;
      rx2[q] = X[(i + 2 < n ? i + 2 : i) * ld + s];
      re[q] = E[o];
      rc[q] = C[o];
      rd[q] = D[o];
      ra[q] = A[o];
      rb[q] = B[o];
      ry[q] = Y[o];
      if (KXB || FIRST) ru0[q] = U0[fo];
      if (KXB) {
        rl2[q] = L2[fo];
        rl1[q] = L1[fo];
        ru1[q] = U1[fo];
      }
    };
    auto use = [&](int q, int64_t kk) {
      const int64_t i = lo + kk;
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
      if (FIRST) {
        bmax = fmax(bmax, fabs(yi));
        if (bad == INT_MAX && bad_pivot(ru0[q])) bad = (int)i;
      }
      if (RES) {
        const double r = yi - ax;
        const double ar = fabs(r);
        if (!isfinite(ar)) nonfinite = true;
        rmax = fmax(rmax, ar);
      }
      if (KXB) {
        const double l2 = (i >= 2) ? rl2[q] : 0.0;
        const double l1 = (i >= 1) ? rl1[q] : 0.0;
        const double u0 = ru0[q];
        const double u1 = (i + 1 < n) ? ru1[q] : 0.0;
        // v = K x + b with K = LU - A
        double kx =
            ((u0 + (i >= 1 ? l1 * u1m1 : 0.0) + (i >= 2 ? l2 * u2m2 : 0.0)) - di) * x0v;
        if (i >= 2) kx = kx + (l2 * u0m2 - ei) * xm2;
        if (i >= 1) kx = kx + (((i >= 2 ? l2 * u1m2 : 0.0) + l1 * u0m1) - ci) * xm1;
        if (i + 1 < n) kx = kx + ((u1 + (i >= 1 ? l1 * u2m1 : 0.0)) - ai) * xp1;
        V[i * lw + s] = kx + yi;
        u0m2 = u0m1;
        u0m1 = u0;
        u1m2 = u1m1;
        u1m1 = u1;
        u2m2 = u2m1;
        u2m1 = bi;
      }
      xm2 = xm1;
      xm1 = x0v;
      x0v = xp1;
      xp1 = xp2;
    };
    stream_rows<PF, false>(hi - lo, fetch, use);
  }
  if (!RES) return;
  const double m = nonfinite ? (double)NAN : rmax;
  s_m[wv][lane] = (unsigned long long)__double_as_longlong(m);
  s_b[wv][lane] = (unsigned long long)__double_as_longlong(bmax);
  s_bad[wv][lane] = bad;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  if (wv == 0) {
    unsigned long long seen = 0;
    if (s < batch && (FIRST || st.active[s] != 0)) {
      unsigned long long mm = 0, bb = 0;
      int br = INT_MAX;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        mm = s_m[w][lane] > mm ? s_m[w][lane] : mm;  // NaN bits compare above every number
        bb = s_b[w][lane] > bb ? s_b[w][lane] : bb;
        br = s_bad[w][lane] < br ? s_bad[w][lane] : br;
      }
      seen |= atomicMax(&st.rmax[s], mm);
      if (FIRST) {
        seen |= atomicMax(&st.bnorm[s], bb);
        seen |= (unsigned long long)(unsigned)atomicMin(&st.badrow[s], br);
      }
    }
    // the arrival waits for every returned value of the wave (vmcnt(0)), so
    // every update of this block is in place before it counts
    __builtin_amdgcn_s_waitcnt(0x0F70);
    if (threadIdx.x == 0 && seen != ~0ull) {
      const unsigned old = atomicAdd(st.arrive, 1u);
      s_last = old == gridDim.x * gridDim.y - 1;
    }
  }
  __syncthreads();
  if (!s_last) return;
  // ---- the last block: Algorithm 1's test for every system ---------------
  for (int64_t q = threadIdx.x; q < batch; q += 256) {
    const double rn = take(&st.rmax[q]);
    if (FIRST) {
      const double bn = __longlong_as_double((long long)st.bnorm[q]);
      if (bn == 0.0) {  // b = 0: x = 0 after no step
        st.zero[q] = 1;
        *st.any_zero = 1;
        iters[q] = 0;
        relres[q] = 0.0;
        info[q] = 0;
        continue;
      }
      if (st.badrow[q] != INT_MAX) {  // an unusable ILU(0) pivot: no step
        iters[q] = 0;
        relres[q] = NAN;
        info[q] = st.badrow[q] + 1;
        continue;
      }
      st.active[q] = 1;
    } else if (!st.active[q]) {
      continue;
    }
    const double bn = __longlong_as_double((long long)st.bnorm[q]);
    const double rr = isfinite(rn) ? rn / bn : (double)NAN;
    if (FIRST) st.relres0[q] = rr;
    int status = 1;
    if (!isfinite(rr))
      status = -2;
    else if (!(rn >= tol * bn))
      status = 0;
    else if (rr > 1e3 * fmax(1.0, st.relres0[q]))
      status = -2;
    else if (k == max_iter)
      status = -1;
    if (status == 1) {
      s_any = 1;
      continue;
    }
    st.active[q] = 0;
    iters[q] = k;
    relres[q] = rr;
    info[q] = status;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_store(st.arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!s_any) *st.done = 1;
  }
}

// x = 0 for the systems whose right-hand side is zero.
__global__ __launch_bounds__(256) void sx_zero_kernel(int64_t n, int64_t batch, int64_t ld,
                                                      double* __restrict__ X, State st) {
  if (!*st.any_zero) return;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n * batch;
       q += (int64_t)gridDim.x * 256) {
    const int64_t s = q % batch, i = q / batch;
    if (st.zero[s]) X[i * ld + s] = 0.0;
  }
}

int grid_for(int64_t work, int block) {
  const int64_t b = (work + block - 1) / block;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

struct Layout {
  size_t v, subst, active, zero, rmax, bnorm, badrow, relres0, done, arrive, any_zero, total;
};

Layout layout(int64_t n, int64_t batch) {
  Layout L;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  size_t o = 0;
  L.v = o;       o = up(o + (size_t)(n * ws_ld(batch)) * 8);
  L.subst = o;   o = up(o + subst_workspace_bytes(n, batch));
  L.active = o;  o = up(o + (size_t)batch * 4);
  L.zero = o;    o = up(o + (size_t)batch * 4);
  L.rmax = o;    o = up(o + (size_t)batch * 8);
  L.bnorm = o;   o = up(o + (size_t)batch * 8);
  L.badrow = o;  o = up(o + (size_t)batch * 4);
  L.relres0 = o; o = up(o + (size_t)batch * 8);
  L.done = o;    o = up(o + 4);
  L.arrive = o;  o = up(o + 4);
  L.any_zero = o; o = up(o + 4);
  L.total = o;
  return L;
}

}  // namespace

bool sip_exact_supported(int64_t n, int64_t batch) { return subst_chunks(n, batch) > 1; }

size_t sip_exact_workspace_bytes(int64_t n, int64_t batch) { return layout(n, batch).total; }

hipError_t launch_sip_exact(int64_t n, int64_t batch, int64_t ld, Diags A, const double* factors,
                            int64_t fld, const double* y, double* x, double tol,
                            int32_t max_iter, int32_t* iters, double* relres, int32_t* info,
                            void* ws, hipStream_t stream) {
  const Layout L = layout(n, batch);
  char* base = static_cast<char*>(ws);
  double* V = reinterpret_cast<double*>(base + L.v);
  double* zws = reinterpret_cast<double*>(base + L.subst);
  State st;
  st.active = reinterpret_cast<int32_t*>(base + L.active);
  st.zero = reinterpret_cast<int32_t*>(base + L.zero);
  st.rmax = reinterpret_cast<unsigned long long*>(base + L.rmax);
  st.bnorm = reinterpret_cast<unsigned long long*>(base + L.bnorm);
  st.badrow = reinterpret_cast<int32_t*>(base + L.badrow);
  st.relres0 = reinterpret_cast<double*>(base + L.relres0);
  st.done = reinterpret_cast<int32_t*>(base + L.done);
  st.arrive = reinterpret_cast<unsigned*>(base + L.arrive);
  st.any_zero = reinterpret_cast<int32_t*>(base + L.any_zero);
  const int64_t lw = ws_ld(batch);
  const int64_t segs = (n + kRB - 1) / kRB;
  const dim3 grid((unsigned)((batch + 63) / 64), (unsigned)((segs + 3) / 4)), block(256);
  hipLaunchKernelGGL(sx_init_kernel, dim3(grid_for(batch, 256)), dim3(256), 0, stream, batch, st);
  hipLaunchKernelGGL(sx_rv_kernel<kFirst>, grid, block, 0, stream, n, batch, ld, A.e, A.c, A.d,
                     A.a, A.b, factors, fld, y, x, V, lw, st, 0, max_iter, tol, iters, relres,
                     info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int32_t k = 1; k <= max_iter; ++k) {
    if (k > 1) {  // v for the systems that failed the test at k - 1
      hipLaunchKernelGGL(sx_rv_kernel<kKxb>, grid, block, 0, stream, n, batch, ld, A.e, A.c,
                         A.d, A.a, A.b, factors, fld, y, x, V, lw, st, k - 1, max_iter, tol,
                         iters, relres, info);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    e = launch_subst_masked(5, n, batch, ld, A, factors, fld, V, lw, x, nullptr, zws, st.active,
                            st.done, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sx_rv_kernel<kResid>, grid, block, 0, stream, n, batch, ld, A.e, A.c,
                       A.d, A.a, A.b, factors, fld, y, x, V, lw, st, k, max_iter, tol, iters,
                       relres, info);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(sx_zero_kernel, dim3(1024), dim3(256), 0, stream, n,
                     batch, ld, x, st);
  return hipGetLastError();
}

}  // namespace bs
