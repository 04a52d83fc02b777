// sip_tile.hip -- the Stone method (SIP) with Hotelling-Bodewig steps for
// both factors, the rows of each system split over many lanes (Veneva &
// Ayriyan, arXiv:1804.09666, Sec. 2 Algorithm 1 and its Remark; Appendix).
//
// One step is x <- x + X_U X_L (b - A x) with X_L, X_U the HB approximate
// inverses after s_L, s_U steps.  Applied to a vector, X_s is 2^s - 1 Jacobi
// sweeps (K = 2^s - 1):
//   lower (X_0 = I):         y_t = y_{t-1} + (v - L y_{t-1}),           y_0 = v
//   upper (X_0 = D_U^{-1}):  z_t = z_{t-1} + (w - U z_{t-1}) / u0,      z_0 = w / u0
// Every sweep is row-parallel and L, U have bandwidth 2, so row i of the
// result depends on x only at rows i - 2 K_L - 2 .. i + 2 K_U + 2.  A block
// therefore owns a tile of "core" rows plus halos of HL = 2 K_L + 2 rows
// before and HR = 2 K_U + 2 rows after it, computes the residual and all the
// sweeps for the whole extended range in registers (one LDS exchange of two
// boundary values per sweep between neighbouring lanes), and writes x for its
// core rows only.  The result at every core row is the one a sweep over the
// whole system produces, with the same operations; the tiling does not change
// it.
//
// One launch per step.  The convergence test must see the whole residual of
// a system, which spans many blocks, so a step reads x_k from one buffer,
// accumulates ||b - A x_k||_inf per system, and always writes the candidate
// x_{k+1} to the other buffer; the last block of the step to finish (an
// arrival counter) then decides, per system, whether x_k was already the
// answer (the candidate is dropped), the step count, the status, and a device
// flag that makes the remaining launches return at once.
#include "bs_internal.h"

// Products and sums may contract into FMAs, the upper sweeps multiply by 1/u0
// (one division per row and step) instead of dividing in every sweep, and the
// sweeps are evaluated in the plain Jacobi form, which is the same polynomial
// with the diagonal terms cancelled:
//   lower: y_t = v - l1 y_{t-1}[i-1] - l2 y_{t-1}[i-2]            (2 FMAs per row)
//   upper: z_t = (w - u1 z_{t-1}[i+1] - u2 z_{t-1}[i+2]) / u0     (2 FMAs, 1 product)
// All three change only the rounding of the iterates.

namespace bs {
namespace {

constexpr int kG = 16;              // systems per block: one 128-byte segment per row
constexpr int kPW = 32;             // lanes per system in a block
constexpr int kM = 8;               // rows per lane
constexpr int kE = kM * kPW;        // rows of a tile including its halos
constexpr int kThreads = kG * kPW;  // 512

__device__ inline void atomic_max_nonneg(unsigned long long* p, double v) {
  atomicMax(p, (unsigned long long)__double_as_longlong(v));  // v >= 0 or NaN
}
__device__ inline double as_double(unsigned long long u) {
  return __longlong_as_double((long long)u);
}

// Per-system state in the workspace.
struct Flags {
  int32_t* active;             // 1 while the system still steps
  int32_t* fin;                // final x: 0 caller's buffer, 1 second buffer, 2 zero
  unsigned long long* accum;   // ||r_k||_inf of the step in flight (bits)
  unsigned long long* bnorm;   // ||b||_inf (bits)
  double* relres0;
  int32_t* done;
  unsigned* arrive;            // blocks of the step in flight that have finished
};

// Algorithm 1's loop test for system s after step k has accumulated
// ||b - A x_k||: returns 1 to keep stepping, else records the outcome.
__device__ inline int sip_status(int64_t s, int32_t k, int32_t max_iter, double tol, Flags fl,
                                 int32_t* __restrict__ iters, double* __restrict__ relres,
                                 int32_t* __restrict__ info) {
  const double rn = as_double(__hip_atomic_exchange(&fl.accum[s], 0ull, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT));
  const double bn = as_double(fl.bnorm[s]);
  const double rr = rn / bn;
  if (k == 0) fl.relres0[s] = rr;
  int status = 1;  // 1: keep stepping
  if (!isfinite(rr))
    status = -2;
  else if (!(rn >= tol * bn))
    status = 0;
  else if (rr > 1e3 * fmax(1.0, fl.relres0[s]))
    status = -2;
  else if (k == max_iter)
    status = -1;
  if (status == 1) return 1;
  fl.active[s] = 0;
  fl.fin[s] = k & 1;  // x_k is in buffer k mod 2
  iters[s] = k;
  relres[s] = rr;
  info[s] = status;
  return 0;
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void sip_step_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ E,
    const double* __restrict__ C, const double* __restrict__ D, const double* __restrict__ A,
    const double* __restrict__ B, const double* __restrict__ F, int64_t fld,
    const double* __restrict__ Y, const double* __restrict__ Xin, double* __restrict__ Xout,
    int KL, int KU, int HL, int RC, int T, Flags fl, int32_t k, int32_t max_iter, double tol,
    int32_t* __restrict__ iters, double* __restrict__ relres, int32_t* __restrict__ info) {
  if (*fl.done) return;
  __shared__ double s_lo[2][kPW][kG][2];  // first two rows of every lane
  __shared__ double s_hi[2][kPW][kG][2];  // last two rows of every lane
  __shared__ unsigned long long s_m[kG];
  __shared__ int s_last, s_any;

  const int tid = threadIdx.x;
  const int g = tid % kG;
  const int j = tid / kG;
  int64_t grp, tile;
  {  // the T tiles of a system group sit on one XCD: halo rows come from its L2
    const int64_t b = blockIdx.x, nblk = gridDim.x;
    if (nblk % (8 * T) == 0) {
      const int64_t k = b / 8, per_xcd = nblk / 8 / T;
      grp = (b % 8) * per_xcd + k / T;
      tile = k % T;
    } else {
      grp = b / T;
      tile = b % T;
    }
  }
  const int64_t s = grp * kG + g;
  const bool live = s < batch && fl.active[s] != 0;
  const int64_t ext0 = tile * RC - HL + (int64_t)j * kM;  // global row of this lane's row 0
  const int64_t plane = n * fld;
  if (tid < kG) s_m[tid] = 0ull;

  double x[kM], e[kM], c[kM], d[kM], a[kM], b[kM], v[kM], l1[kM], l2[kM], u0[kM], u1[kM];
#pragma unroll
  for (int r = 0; r < kM; ++r) {
    const int64_t i = ext0 + r;
    const bool in = live && i >= 0 && i < n;
    const int64_t o = in ? i * ld + s : 0;
    const int64_t fo = in ? i * fld + s : 0;
    x[r] = in ? Xin[o] : 0.0;
    d[r] = in ? D[o] : 1.0;
    v[r] = in ? Y[o] : 0.0;
    c[r] = (in && i >= 1) ? C[o] : 0.0;
    a[r] = (in && i <= n - 2) ? A[o] : 0.0;
    e[r] = (in && i >= 2) ? E[o] : 0.0;
    b[r] = (in && i <= n - 3) ? B[o] : 0.0;
    l2[r] = (in && i >= 2) ? F[fo] : 0.0;
    l1[r] = (in && i >= 1) ? F[plane + fo] : 0.0;
    u0[r] = in ? F[2 * plane + fo] : 1.0;
    u1[r] = (in && i <= n - 2) ? F[3 * plane + fo] : 0.0;
  }

  // ---- residual r = b - A x over the extended range (v holds r) -----------
  s_lo[0][j][g][0] = x[0];
  s_lo[0][j][g][1] = x[1];
  s_hi[0][j][g][0] = x[kM - 2];
  s_hi[0][j][g][1] = x[kM - 1];
  __syncthreads();
  {
    const double xm2 = j > 0 ? s_hi[0][j - 1][g][0] : 0.0;
    const double xm1 = j > 0 ? s_hi[0][j - 1][g][1] : 0.0;
    const double xp1 = j < kPW - 1 ? s_lo[0][j + 1][g][0] : 0.0;
    const double xp2 = j < kPW - 1 ? s_lo[0][j + 1][g][1] : 0.0;
    double m = 0.0;
#pragma unroll
    for (int r = 0; r < kM; ++r) {
      const double x_m2 = r >= 2 ? x[r - 2] : (r == 1 ? xm1 : xm2);
      const double x_m1 = r >= 1 ? x[r - 1] : xm1;
      const double x_p1 = r + 1 < kM ? x[r + 1] : xp1;
      const double x_p2 = r + 2 < kM ? x[r + 2] : (r + 2 == kM ? xp1 : xp2);
      double ax = d[r] * x[r];
      ax = ax + e[r] * x_m2;
      ax = ax + c[r] * x_m1;
      ax = ax + a[r] * x_p1;
      ax = ax + b[r] * x_p2;
      v[r] = v[r] - ax;
      const int64_t q = (int64_t)j * kM + r;  // row within the extended tile
      const int64_t i = ext0 + r;
      if (q >= HL && q < HL + RC && i < n) {
        const double ar = fabs(v[r]);
        m = (ar > m || ar != ar) ? ar : m;
      }
    }
    if (live && m != 0.0) atomicMax(&s_m[g], (unsigned long long)__double_as_longlong(m));
  }

  // ---- y = X_L r: K_L lower sweeps, rows descending within the lane ------
  double y[kM];
#pragma unroll
  for (int r = 0; r < kM; ++r) y[r] = v[r];
  for (int t = 1; t <= KL; ++t) {
    const int p = t & 1;
    s_hi[p][j][g][0] = y[kM - 2];
    s_hi[p][j][g][1] = y[kM - 1];
    __syncthreads();
    const double ym2 = j > 0 ? s_hi[p][j - 1][g][0] : 0.0;
    const double ym1 = j > 0 ? s_hi[p][j - 1][g][1] : 0.0;
#pragma unroll
    for (int r = kM - 1; r >= 0; --r) {
      const double y_m1 = r >= 1 ? y[r - 1] : ym1;
      const double y_m2 = r >= 2 ? y[r - 2] : (r == 1 ? ym1 : ym2);
      double ty = v[r];
      ty = ty - l1[r] * y_m1;
      ty = ty - l2[r] * y_m2;
      y[r] = ty;
    }
  }

  // ---- z = X_U y: K_U upper sweeps, rows ascending within the lane -------
  double z[kM], ru[kM];
#pragma unroll
  for (int r = 0; r < kM; ++r) {
    ru[r] = 1.0 / u0[r];
    z[r] = y[r] * ru[r];
  }
  for (int t = 1; t <= KU; ++t) {
    const int p = t & 1;
    s_lo[p][j][g][0] = z[0];
    s_lo[p][j][g][1] = z[1];
    __syncthreads();
    const double zp1 = j < kPW - 1 ? s_lo[p][j + 1][g][0] : 0.0;
    const double zp2 = j < kPW - 1 ? s_lo[p][j + 1][g][1] : 0.0;
#pragma unroll
    for (int r = 0; r < kM; ++r) {
      const double z_p1 = r + 1 < kM ? z[r + 1] : zp1;
      const double z_p2 = r + 2 < kM ? z[r + 2] : (r + 2 == kM ? zp1 : zp2);
      double ty = y[r];
      ty = ty - u1[r] * z_p1;
      ty = ty - b[r] * z_p2;
      z[r] = ty * ru[r];
    }
  }

  // ---- candidate x_{k+1} for the core rows; residual norm of x_k ---------
  if (live) {
#pragma unroll
    for (int r = 0; r < kM; ++r) {
      const int64_t q = (int64_t)j * kM + r;
      const int64_t i = ext0 + r;
      if (q >= HL && q < HL + RC && i < n) Xout[i * ld + s] = x[r] + z[r];
    }
  }
  __syncthreads();
  // ---- the last block of the step applies the test for every system ------
  if (tid < 64) {  // wave 0: this block's maxima, then its arrival
    unsigned long long seen = 0;
    if (j == 0 && live) seen = atomicMax(&fl.accum[s], s_m[g]);
    // the arrival waits for the returned maxima (one instruction for the
    // wave): every maximum of this block is in place before it counts
    if (tid == 0 && seen != ~0ull) {
      const unsigned old = atomicAdd(fl.arrive, 1u);
      s_last = old == gridDim.x - 1;
      s_any = 0;
    }
  }
  __syncthreads();
  if (!s_last) return;
  for (int64_t q = tid; q < batch; q += kThreads)
    if (fl.active[q] && sip_status(q, k, max_iter, tol, fl, iters, relres, info)) s_any = 1;
  __syncthreads();
  if (tid == 0) {
    __hip_atomic_store(fl.arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!s_any) *fl.done = 1;
  }
}

// ||b||_inf per system (bits into bnorm, zeroed by init_kernel).
__global__ __launch_bounds__(256) void bnorm_kernel(int64_t n, int64_t batch, int64_t ld,
                                                    const double* __restrict__ Y, Flags fl) {
  const int64_t parts = (int64_t)gridDim.x * 256 / batch > 0 ? (int64_t)gridDim.x * 256 / batch : 1;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < batch * parts;
       q += (int64_t)gridDim.x * 256) {
    const int64_t s = q % batch, part = q / batch;
    double m = 0.0;
    constexpr int U = 8;  // loads in flight per thread
    for (int64_t i = part; i < n; i += U * parts) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = i + u * parts;
        v[u] = r < n ? fabs(Y[r * ld + s]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) m = (v[u] > m || v[u] != v[u]) ? v[u] : m;
    }
    if (m != 0.0) atomic_max_nonneg(&fl.bnorm[s], m);
  }
}

__global__ void init_kernel(int64_t batch, Flags fl, int32_t* iters, double* relres,
                            int32_t* info, int own_factors) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < batch;
       s += (int64_t)gridDim.x * blockDim.x) {
    fl.bnorm[s] = 0ull;
    fl.accum[s] = 0ull;
    fl.active[s] = 0;
    fl.fin[s] = 0;
    fl.relres0[s] = 0.0;
    iters[s] = 0;
    relres[s] = 0.0;
    if (!own_factors) info[s] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *fl.done = 0;
    *fl.arrive = 0u;
  }
}

// After the factorization and ||b||: which systems step at all.
__global__ void start_kernel(int64_t batch, Flags fl, int32_t* info) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < batch;
       s += (int64_t)gridDim.x * blockDim.x) {
    if (info[s] != 0) continue;  // unusable ILU(0) pivot: no step, x untouched
    if (fl.bnorm[s] == 0ull) {
      fl.fin[s] = 2;  // b = 0: x = 0, no step
      continue;
    }
    fl.active[s] = 1;
  }
}

// The answer of every system into the caller's x.
__global__ __launch_bounds__(256) void finish_kernel(int64_t n, int64_t batch, int64_t ld,
                                                     const double* __restrict__ X1,
                                                     double* __restrict__ X, Flags fl) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n * batch;
       q += (int64_t)gridDim.x * 256) {
    const int64_t s = q % batch, i = q / batch;
    const int f = fl.fin[s];
    if (f == 1) X[i * ld + s] = X1[i * ld + s];
    else if (f == 2) X[i * ld + s] = 0.0;
  }
}

int grid_for(int64_t work, int block) {
  const int64_t b = (work + block - 1) / block;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

struct Layout {
  size_t x1, active, fin, accum, bnorm, relres0, done, arrive, total;
};

Layout layout(int64_t n, int64_t batch, int64_t ld) {
  Layout L;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  size_t o = 0;
  L.x1 = o;      o = up(o + (size_t)(n * ld) * 8);
  L.active = o;  o = up(o + (size_t)batch * 4);
  L.fin = o;     o = up(o + (size_t)batch * 4);
  L.accum = o;   o = up(o + (size_t)batch * 8);
  L.bnorm = o;   o = up(o + (size_t)batch * 8);
  L.relres0 = o; o = up(o + (size_t)batch * 8);
  L.done = o;    o = up(o + 4);
  L.arrive = o;  o = up(o + 4);
  L.total = o;
  return L;
}

}  // namespace

bool sip_tile_supported(int64_t n, int32_t sL, int32_t sU) {
  if (sL < 0 || sU < 0 || sL > 6 || sU > 6) return false;
  const int64_t KL = (int64_t(1) << sL) - 1, KU = (int64_t(1) << sU) - 1;
  if (KL + 1 >= n || KU + 1 >= n) return false;  // HB exact: substitution instead
  return kE - (2 * KL + 2) - (2 * KU + 2) >= 64;
}

size_t sip_tile_workspace_bytes(int64_t n, int64_t batch, int64_t ld) {
  return layout(n, batch, ld).total;
}

hipError_t launch_sip_tile(int64_t n, int64_t batch, int64_t ld, Diags A, const double* factors,
                           int64_t fld, bool own_factors, const double* y, double* x, double tol,
                           int32_t max_iter, int32_t sL, int32_t sU, int32_t* iters,
                           double* relres, int32_t* info, void* ws, hipStream_t st) {
  const Layout L = layout(n, batch, ld);
  char* base = static_cast<char*>(ws);
  double* x1 = reinterpret_cast<double*>(base + L.x1);
  Flags fl;
  fl.active = reinterpret_cast<int32_t*>(base + L.active);
  fl.fin = reinterpret_cast<int32_t*>(base + L.fin);
  fl.accum = reinterpret_cast<unsigned long long*>(base + L.accum);
  fl.bnorm = reinterpret_cast<unsigned long long*>(base + L.bnorm);
  fl.relres0 = reinterpret_cast<double*>(base + L.relres0);
  fl.done = reinterpret_cast<int32_t*>(base + L.done);
  fl.arrive = reinterpret_cast<unsigned*>(base + L.arrive);
  const int KL = (1 << sL) - 1, KU = (1 << sU) - 1;
  const int HL = 2 * KL + 2, HR = 2 * KU + 2;
  const int RC = kE - HL - HR;
  const int64_t T = (n + RC - 1) / RC;
  const int64_t groups = (batch + kG - 1) / kG;

  hipLaunchKernelGGL(init_kernel, dim3(grid_for(batch, 256)), dim3(256), 0, st, batch, fl, iters,
                     relres, info, (int)own_factors);
  // about 32 rows per thread: few atomics per system, enough blocks in flight
  hipLaunchKernelGGL(bnorm_kernel, dim3(grid_for(batch * ((n + 31) / 32), 256)), dim3(256), 0, st,
                     n, batch, ld, y, fl);
  hipLaunchKernelGGL(start_kernel, dim3(grid_for(batch, 256)), dim3(256), 0, st, batch, fl, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int32_t k = 0; k <= max_iter; ++k) {
    const double* xin = (k & 1) ? x1 : x;
    double* xout = (k & 1) ? x : x1;
    hipLaunchKernelGGL(sip_step_kernel, dim3((unsigned)(groups * T)), dim3(kThreads), 0, st, n,
                       batch, ld, A.e, A.c, A.d, A.a, A.b, factors, fld, y, xin, xout, KL, KU, HL,
                       RC, (int)T, fl, k, max_iter, tol, iters, relres, info);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(finish_kernel, dim3(grid_for(n * batch, 256)), dim3(256), 0, st, n, batch,
                     ld, x1, x, fl);
  return hipGetLastError();
}

}  // namespace bs
