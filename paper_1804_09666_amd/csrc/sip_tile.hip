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
// before and HR = 2 K_U + 2 rows after it per step, computes the residual and
// all the sweeps for the whole extended range in registers (one LDS exchange
// of two boundary values per sweep between neighbouring lanes), and writes x
// for its core rows only.  The result at every core row is the one a sweep
// over the whole system produces, with the same operations; the tiling does
// not change it.
//
// One launch takes two steps (halos 2 HL and 2 HR; the rows of A, b and the
// factors are loaded once for both), or one where the doubled halos leave
// too small a core.  The convergence test must see the whole residual of a
// system, which spans many blocks, so a launch reads x_k from one buffer,
// accumulates ||b - A x_k||_inf (and ||b - A x_{k+1}||_inf) per system, and
// always writes the candidates x_{k+1} (and x_{k+2}) to the next buffers; the
// last block of the launch to finish (an arrival counter) then decides, per
// system, which iterate is the answer, the step count, the status, and a
// device flag that makes the remaining launches return at once.
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

constexpr int kG = 16;   // systems per block: one 128-byte segment per row
constexpr int kE = 256;  // rows of a tile including its halos
// Tile shapes (rows per lane KM x lanes per system KPW = kE):
//   one step per launch:  8 x 32, 512 threads at two waves per SIMD;
//   two steps per launch: 16 x 16, 256 threads at one wave per SIMD (the rows
//     of A and the right-hand side stay live through the first step).
constexpr int kMaxSteps = 3;  // steps per launch at most
constexpr int kZero = 7;      // fin: the answer is x = 0 (b = 0)

__device__ inline void atomic_max_nonneg(unsigned long long* p, double v) {
  atomicMax(p, (unsigned long long)__double_as_longlong(v));  // v >= 0 or NaN
}
__device__ inline double as_double(unsigned long long u) {
  return __longlong_as_double((long long)u);
}

// Per-system state in the workspace.
struct Flags {
  int32_t* active;               // 1 while the system still steps
  int32_t* fin;                  // buffer holding the answer (0 = caller's x), or kZero
  unsigned long long* accum[kMaxSteps];  // ||r_k||_inf, ||r_{k+1}||_inf, ... of the launch in flight (bits)
  unsigned long long* bnorm;     // ||b||_inf (bits)
  double* relres0;
  int32_t* done;
  unsigned* arrive;              // blocks of the launch in flight that have finished
};

// Algorithm 1's loop test for system s at step count k with rn = ||b - A x_k||:
// returns 1 to keep stepping, else records the outcome (x_k, in buffer
// `buf`, is the answer).
__device__ inline int sip_test(int64_t s, int32_t k, double rn, int buf, int32_t max_iter,
                               double tol, Flags fl, int32_t* __restrict__ iters,
                               double* __restrict__ relres, int32_t* __restrict__ info) {
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
  fl.fin[s] = buf;
  iters[s] = k;
  relres[s] = rr;
  info[s] = status;
  return 0;
}

__device__ inline double take(unsigned long long* acc, int64_t s) {
  return as_double(__hip_atomic_exchange(&acc[s], 0ull, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT));
}

// First and last two rows of every lane, double-buffered by sweep parity.
template <int KPW>
struct Halo {
  double lo[2][KPW][kG][2];
  double hi[2][KPW][kG][2];
};

// v = w - A x over the lane's rows (the first and last two rows of the tile
// see zero outside it); returns max |v| over tile rows [c0, c1) inside the
// matrix.  Starts with a barrier-protected exchange of x's tip rows.
template <int KM, int KPW>
__device__ inline double residual(const double (&x)[KM], const double (&e)[KM],
                                  const double (&c)[KM], const double (&d)[KM],
                                  const double (&a)[KM], const double (&b)[KM],
                                  const double (&w)[KM], double (&v)[KM], Halo<KPW>& H, int j,
                                  int g, int64_t ext0, int c0, int c1, int64_t n) {
  H.lo[0][j][g][0] = x[0];
  H.lo[0][j][g][1] = x[1];
  H.hi[0][j][g][0] = x[KM - 2];
  H.hi[0][j][g][1] = x[KM - 1];
  __syncthreads();
  const double xm2 = j > 0 ? H.hi[0][j - 1][g][0] : 0.0;
  const double xm1 = j > 0 ? H.hi[0][j - 1][g][1] : 0.0;
  const double xp1 = j < KPW - 1 ? H.lo[0][j + 1][g][0] : 0.0;
  const double xp2 = j < KPW - 1 ? H.lo[0][j + 1][g][1] : 0.0;
  double m = 0.0;
#pragma unroll
  for (int r = 0; r < KM; ++r) {
    const double x_m2 = r >= 2 ? x[r - 2] : (r == 1 ? xm1 : xm2);
    const double x_m1 = r >= 1 ? x[r - 1] : xm1;
    const double x_p1 = r + 1 < KM ? x[r + 1] : xp1;
    const double x_p2 = r + 2 < KM ? x[r + 2] : (r + 2 == KM ? xp1 : xp2);
    double ax = d[r] * x[r];
    ax = ax + e[r] * x_m2;
    ax = ax + c[r] * x_m1;
    ax = ax + a[r] * x_p1;
    ax = ax + b[r] * x_p2;
    v[r] = w[r] - ax;
    const int q = j * KM + r;  // row within the extended tile
    if (q >= c0 && q < c1 && ext0 + r < n) {
      const double ar = fabs(v[r]);
      m = (ar > m || ar != ar) ? ar : m;
    }
  }
  return m;
}

// y = X_L v: K_L lower sweeps, rows descending within the lane.
template <int KM, int KPW>
__device__ inline void lower_sweeps(int KL, const double (&v)[KM], const double (&l1)[KM],
                                    const double (&l2)[KM], double (&y)[KM], Halo<KPW>& H, int j,
                                    int g) {
#pragma unroll
  for (int r = 0; r < KM; ++r) y[r] = v[r];
  for (int t = 1; t <= KL; ++t) {
    const int p = t & 1;
    H.hi[p][j][g][0] = y[KM - 2];
    H.hi[p][j][g][1] = y[KM - 1];
    __syncthreads();
    const double ym2 = j > 0 ? H.hi[p][j - 1][g][0] : 0.0;
    const double ym1 = j > 0 ? H.hi[p][j - 1][g][1] : 0.0;
#pragma unroll
    for (int r = KM - 1; r >= 0; --r) {
      const double y_m1 = r >= 1 ? y[r - 1] : ym1;
      const double y_m2 = r >= 2 ? y[r - 2] : (r == 1 ? ym1 : ym2);
      double ty = v[r];
      ty = ty - l1[r] * y_m1;
      ty = ty - l2[r] * y_m2;
      y[r] = ty;
    }
  }
}

// z = X_U w: K_U upper sweeps, rows ascending within the lane (ru = 1/u0).
template <int KM, int KPW>
__device__ inline void upper_sweeps(int KU, const double (&w)[KM], const double (&u1)[KM],
                                    const double (&u2)[KM], const double (&ru)[KM],
                                    double (&z)[KM], Halo<KPW>& H, int j, int g) {
#pragma unroll
  for (int r = 0; r < KM; ++r) z[r] = w[r] * ru[r];
  for (int t = 1; t <= KU; ++t) {
    const int p = t & 1;
    H.lo[p][j][g][0] = z[0];
    H.lo[p][j][g][1] = z[1];
    __syncthreads();
    const double zp1 = j < KPW - 1 ? H.lo[p][j + 1][g][0] : 0.0;
    const double zp2 = j < KPW - 1 ? H.lo[p][j + 1][g][1] : 0.0;
#pragma unroll
    for (int r = 0; r < KM; ++r) {
      const double z_p1 = r + 1 < KM ? z[r + 1] : zp1;
      const double z_p2 = r + 2 < KM ? z[r + 2] : (r + 2 == KM ? zp1 : zp2);
      double ty = w[r];
      ty = ty - u1[r] * z_p1;
      ty = ty - u2[r] * z_p2;
      z[r] = ty * ru[r];
    }
  }
}

// The buffers a launch writes x_{k+1}, ..., x_{k+NS} to.
struct Outs {
  double* p[kMaxSteps];
};

// NS steps of Algorithm 1 (1 <= NS <= 3) for every system in one launch.
// Launch k reads x_k from buffer k mod (NS + 1) and writes x_{k+1}, ...,
// x_{k+NS} to the next buffers; the tile has halos of NS * HL rows before
// and NS * HR after its RC core rows, which is what NS steps need for every
// core row to get exactly the value of steps over the whole system.
// The last block of the launch to finish (an arrival counter) applies the
// test at k, k + 1, ... in turn for every system still stepping.
template <int KM, int KPW, int NS, int WPE>
__global__ __launch_bounds__(kG * KPW) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void sip_step_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ E,
    const double* __restrict__ C, const double* __restrict__ D, const double* __restrict__ A,
    const double* __restrict__ B, const double* __restrict__ F, int64_t fld,
    const double* __restrict__ Y, const double* __restrict__ Xin, Outs xo,
    int KL, int KU, int HL, int RC, int T, Flags fl, int32_t k,
    int32_t max_iter, double tol, int32_t* __restrict__ iters, double* __restrict__ relres,
    int32_t* __restrict__ info) {
  static_assert(KM * KPW == kE && KM >= 4 && NS >= 1 && NS <= kMaxSteps, "shape");
  constexpr int kThreads = kG * KPW;
  if (*fl.done) return;
  __shared__ Halo<KPW> H;
  __shared__ unsigned long long s_m[NS][kG];
  __shared__ int s_last, s_any;

  const int tid = threadIdx.x;
  const int g = tid % kG;
  const int j = tid / kG;
  int64_t grp, tile;
  {  // the T tiles of a system group sit on one XCD: halo rows come from its L2
    const int64_t b = blockIdx.x, nblk = gridDim.x;
    if (nblk % (8 * T) == 0) {
      const int64_t q = b / 8, per_xcd = nblk / 8 / T;
      grp = (b % 8) * per_xcd + q / T;
      tile = q % T;
    } else {
      grp = b / T;
      tile = b % T;
    }
  }
  const int64_t s = grp * kG + g;
  const bool live = s < batch && fl.active[s] != 0;
  const int c0 = NS * HL, c1 = NS * HL + RC;            // core rows of the tile
  const int64_t ext0 = tile * RC - c0 + (int64_t)j * KM;  // global row of this lane's row 0
  const int64_t plane = n * fld;
  if (tid < kG) {
#pragma unroll
    for (int u = 0; u < NS; ++u) s_m[u][tid] = 0ull;
  }

  double x[KM], e[KM], c[KM], d[KM], a[KM], b[KM], w[KM], l1[KM], l2[KM], u0[KM], u1[KM];
#pragma unroll
  for (int r = 0; r < KM; ++r) {
    const int64_t i = ext0 + r;
    const bool in = live && i >= 0 && i < n;
    const int64_t o = in ? i * ld + s : 0;
    const int64_t fo = in ? i * fld + s : 0;
    x[r] = in ? Xin[o] : 0.0;
    d[r] = in ? D[o] : 1.0;
    w[r] = in ? Y[o] : 0.0;
    c[r] = (in && i >= 1) ? C[o] : 0.0;
    a[r] = (in && i <= n - 2) ? A[o] : 0.0;
    e[r] = (in && i >= 2) ? E[o] : 0.0;
    b[r] = (in && i <= n - 3) ? B[o] : 0.0;
    l2[r] = (in && i >= 2) ? F[fo] : 0.0;
    l1[r] = (in && i >= 1) ? F[plane + fo] : 0.0;
    u0[r] = in ? F[2 * plane + fo] : 1.0;
    u1[r] = (in && i <= n - 2) ? F[3 * plane + fo] : 0.0;
  }
  double ru[KM];
#pragma unroll
  for (int r = 0; r < KM; ++r) ru[r] = 1.0 / u0[r];

  double v[KM], y[KM], z[KM];
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    if (u > 0) __syncthreads();  // every read of the previous step's exchanges is done
    const double m = residual<KM, KPW>(x, e, c, d, a, b, w, v, H, j, g, ext0, c0, c1, n);
    {  // max over the wave's lanes of each system (lanes g, g + kG, ...: non-negative
       // doubles, NaN included, order like their bit patterns), then one LDS
       // atomic per system and wave
      unsigned long long mb = live ? (unsigned long long)__double_as_longlong(m) : 0ull;
#pragma unroll
      for (int off = kG; off < 64; off <<= 1) {
        const unsigned long long o = __shfl_xor(mb, off, 64);
        mb = o > mb ? o : mb;
      }
      if ((tid & 63) < kG && mb != 0ull) atomicMax(&s_m[u][g], mb);
    }
    lower_sweeps<KM, KPW>(KL, v, l1, l2, y, H, j, g);
    upper_sweeps<KM, KPW>(KU, y, u1, b, ru, z, H, j, g);
#pragma unroll
    for (int r = 0; r < KM; ++r) x[r] = x[r] + z[r];
    if (live) {  // x_{k+u+1} at the core rows
      double* __restrict__ Xo = xo.p[u];
#pragma unroll
      for (int r = 0; r < KM; ++r) {
        const int q = j * KM + r;
        const int64_t i = ext0 + r;
        if (q >= c0 && q < c1 && i < n) Xo[i * ld + s] = x[r];
      }
    }
  }
  __syncthreads();
  // ---- the last block of the launch applies the tests for every system ---
  if (tid < 64) {  // wave 0: this block's maxima, then its arrival
    unsigned long long seen = 0;
    if (j == 0 && live) {
#pragma unroll
      for (int u = 0; u < NS; ++u) seen |= atomicMax(&fl.accum[u][s], s_m[u][g]);
    }
    // the arrival waits for the returned maxima (one instruction for the
    // wave each): every maximum of this block is in place before it counts
    if (tid == 0 && seen != ~0ull) {
      const unsigned old = atomicAdd(fl.arrive, 1u);
      s_last = old == gridDim.x - 1;
      s_any = 0;
    }
  }
  __syncthreads();
  if (!s_last) return;
  for (int64_t q = tid; q < batch; q += kThreads) {
    if (!fl.active[q]) continue;
    double r[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) r[u] = take(fl.accum[u], q);
    // x_j sits in buffer j mod (NS + 1); a system that passes the test at
    // k + u has k + u < max_iter, so k + u + 1 is a step it may still take
    int keep = 1;
#pragma unroll
    for (int u = 0; u < NS; ++u)
      if (keep)
        keep = sip_test(q, k + u, r[u], (k + u) % (NS + 1), max_iter, tol, fl, iters, relres,
                        info);
    if (keep) s_any = 1;
  }
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
#pragma unroll
    for (int u = 0; u < kMaxSteps; ++u) fl.accum[u][s] = 0ull;
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
      fl.fin[s] = kZero;  // b = 0: x = 0, no step
      continue;
    }
    fl.active[s] = 1;
  }
}

// The answer of every system into the caller's x (buffer 0).
__global__ __launch_bounds__(256) void finish_kernel(int64_t n, int64_t batch, int64_t ld,
                                                     Outs more, double* __restrict__ X,
                                                     Flags fl) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n * batch;
       q += (int64_t)gridDim.x * 256) {
    const int64_t s = q % batch, i = q / batch;
    const int f = fl.fin[s];  // buffers 1.. are more.p[0..]
    if (f >= 1 && f <= kMaxSteps) X[i * ld + s] = more.p[f - 1][i * ld + s];
    else if (f == kZero) X[i * ld + s] = 0.0;
  }
}

int grid_for(int64_t work, int block) {
  const int64_t b = (work + block - 1) / block;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

struct Layout {
  size_t x[kMaxSteps], active, fin, accum[kMaxSteps], bnorm, relres0, done, arrive, total;
};

Layout layout(int64_t n, int64_t batch, int64_t ld) {
  Layout L;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  size_t o = 0;
  for (int u = 0; u < kMaxSteps; ++u) {  // x buffers 1..kMaxSteps
    L.x[u] = o;
    o = up(o + (size_t)(n * ld) * 8);
  }
  L.active = o;  o = up(o + (size_t)batch * 4);
  L.fin = o;     o = up(o + (size_t)batch * 4);
  for (int u = 0; u < kMaxSteps; ++u) {
    L.accum[u] = o;
    o = up(o + (size_t)batch * 8);
  }
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
                           double* relres, int32_t* info, void* ws, int steps_per_launch,
                           hipStream_t st) {
  const Layout L = layout(n, batch, ld);
  char* base = static_cast<char*>(ws);
  double* buf[kMaxSteps + 1] = {x};
  Outs more;
  for (int u = 0; u < kMaxSteps; ++u) more.p[u] = buf[u + 1] = reinterpret_cast<double*>(base + L.x[u]);
  Flags fl;
  fl.active = reinterpret_cast<int32_t*>(base + L.active);
  fl.fin = reinterpret_cast<int32_t*>(base + L.fin);
  for (int u = 0; u < kMaxSteps; ++u)
    fl.accum[u] = reinterpret_cast<unsigned long long*>(base + L.accum[u]);
  fl.bnorm = reinterpret_cast<unsigned long long*>(base + L.bnorm);
  fl.relres0 = reinterpret_cast<double*>(base + L.relres0);
  fl.done = reinterpret_cast<int32_t*>(base + L.done);
  fl.arrive = reinterpret_cast<unsigned*>(base + L.arrive);
  const int KL = (1 << sL) - 1, KU = (1 << sU) - 1;
  const int HL = 2 * KL + 2, HR = 2 * KU + 2;
  // three steps per launch where their halos leave a core of 160 rows or
  // more, two where they leave 64, else one
  int NS = 1;
  if (steps_per_launch >= 3 && kE - 3 * (HL + HR) >= 160)
    NS = 3;
  else if (steps_per_launch >= 2 && kE - 2 * (HL + HR) >= 64)
    NS = 2;
  const int RC = kE - NS * (HL + HR);
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
  const dim3 grid((unsigned)(groups * T)), block(kG * 32);
  for (int32_t k = 0; k <= max_iter; k += NS) {
    const double* xin = buf[k % (NS + 1)];
    Outs xo{};
    for (int u = 0; u < NS; ++u) xo.p[u] = buf[(k + 1 + u) % (NS + 1)];
    if (NS == 3)
      hipLaunchKernelGGL((sip_step_kernel<8, 32, 3, 2>), grid, block, 0, st, n, batch, ld, A.e,
                         A.c, A.d, A.a, A.b, factors, fld, y, xin, xo, KL, KU, HL, RC, (int)T, fl,
                         k, max_iter, tol, iters, relres, info);
    else if (NS == 2)
      hipLaunchKernelGGL((sip_step_kernel<8, 32, 2, 2>), grid, block, 0, st, n, batch, ld, A.e,
                         A.c, A.d, A.a, A.b, factors, fld, y, xin, xo, KL, KU, HL, RC, (int)T, fl,
                         k, max_iter, tol, iters, relres, info);
    else
      hipLaunchKernelGGL((sip_step_kernel<8, 32, 1, 2>), grid, block, 0, st, n, batch, ld, A.e,
                         A.c, A.d, A.a, A.b, factors, fld, y, xin, xo, KL, KU, HL, RC, (int)T, fl,
                         k, max_iter, tol, iters, relres, info);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(finish_kernel, dim3(grid_for(n * batch, 256)), dim3(256), 0, st, n, batch,
                     ld, more, x, fl);
  return hipGetLastError();
}

}  // namespace bs
