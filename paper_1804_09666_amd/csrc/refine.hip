// refine.hip -- low-precision direct solves with FP64 iterative refinement.
//
//   r = b, x = 0
//   repeat: solve A d = r in low precision;  x += d;  r = b - A x (FP64)
//   until ||r||_inf < tol ||b||_inf per system (masked), or max_steps.
// Two ways to solve in low precision:
//  - compact (the sweep's systems, n <= 4096, the default FP32 state): the
//    split kernel with FP32 per-row state reads the FP64 A and r directly (no
//    FP32 copy of A is made) and adds d into x as it stores it; the residual
//    pass writes r in FP64 and, on the first pass, takes ||b||.
//  - FP32 storage (longer systems, or BS_OPT_F32_STATE = 0): A32 = fl32(A)
//    once, then solve A32 d = fl32(r) with the FP32-storage kernels and add d
//    in a separate pass.
// All steps run on the stream without host round-trips: a device flag makes
// the remaining launches return at once when every system has converged.
#include "bs_internal.h"

namespace bs {
namespace {

constexpr int kBlock = 256;

__device__ inline void atomic_max_nonneg(unsigned long long* p, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

__device__ inline double as_double(unsigned long long u) {
  return __longlong_as_double((long long)u);
}

struct Planes {
  const double* p[5];
};

// A32 = fl32(A) for every plane, r32 = fl32(b), x = 0, |b|_inf per system.
// Work item q = (s, part) walks rows part, part + P, ... of system s and
// folds |b| into one maximum before its single atomic.
__global__ __launch_bounds__(kBlock) void setup_kernel(
    int64_t n, int64_t batch, int64_t ld, int nplanes, Planes pl, float* __restrict__ a32,
    const double* __restrict__ b, float* __restrict__ r32, double* __restrict__ x,
    unsigned long long* __restrict__ bmax, int64_t parts) {
  const int64_t plane = n * ld;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < batch * parts;
       q += (int64_t)gridDim.x * kBlock) {
    const int64_t s = q % batch, part = q / batch;
    double m = 0.0;
    for (int64_t i = part; i < n; i += parts) {
      const int64_t o = i * ld + s;
      for (int k = 0; k < nplanes; ++k) a32[k * plane + o] = (float)pl.p[k][o];
      const double bv = b[o];
      r32[o] = (float)bv;
      x[o] = 0.0;
      const double av = fabs(bv);
      m = (av > m || av != av) ? av : m;
    }
    atomic_max_nonneg(&bmax[s], m);
  }
}

// x += d for the systems still refining.
__global__ __launch_bounds__(kBlock) void update_kernel(
    int64_t n, int64_t batch, int64_t ld, const float* __restrict__ d, double* __restrict__ x,
    const int32_t* __restrict__ active, const int32_t* __restrict__ done) {
  if (*done) return;
  const int64_t total = n * batch;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlock) {
    const int64_t s = q % batch, i = q / batch;
    if (!active[s]) continue;
    const int64_t o = i * ld + s;
    x[o] += (double)d[o];
  }
}

// r = b - A x in FP64 (row i of system s reads x at rows i-2 .. i+2),
// r32 = fl32(r), |r|_inf per system.  Work item q = (s, part) walks rows
// part, part + P, ... of system s; consecutive items are consecutive
// systems, so each row access of a wave is one contiguous segment.
// TR: type of the stored residual (float for the FP32-storage solve, double
// for the compact one).  BNORM: also |b|_inf into bmax.  act (nullable):
// systems with act[s] == 0 are skipped.
template <int KIND, typename TR, bool BNORM>
__global__ __launch_bounds__(kBlock) void residual_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ E,
    const double* __restrict__ C, const double* __restrict__ D, const double* __restrict__ A,
    const double* __restrict__ B, const double* __restrict__ b, const double* __restrict__ x,
    TR* __restrict__ r32, unsigned long long* __restrict__ rmax, int64_t parts,
    const int32_t* __restrict__ done, unsigned long long* __restrict__ bmax,
    const int32_t* __restrict__ act) {
  if (*done) return;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < batch * parts;
       q += (int64_t)gridDim.x * kBlock) {
    const int64_t s = q % batch, part = q / batch;
    if (act != nullptr && !act[s]) continue;
    double m = 0.0, mb = 0.0;
    for (int64_t i = part; i < n; i += parts) {
      const int64_t o = i * ld + s;
      double ax = D[o] * x[o];
      if (i >= 1) ax = fma(C[o], x[o - ld], ax);
      if (i + 1 < n) ax = fma(A[o], x[o + ld], ax);
      if (KIND == 5) {
        if (i >= 2) ax = fma(E[o], x[o - 2 * ld], ax);
        if (i + 2 < n) ax = fma(B[o], x[o + 2 * ld], ax);
      }
      const double bv = b[o];
      const double r = bv - ax;
      r32[o] = (TR)r;
      const double ar = fabs(r);
      m = (ar > m || ar != ar) ? ar : m;  // a NaN residual stays visible
      if (BNORM) {
        const double ab = fabs(bv);
        mb = (ab > mb || ab != ab) ? ab : mb;
      }
    }
    atomic_max_nonneg(&rmax[s], m);
    if (BNORM) atomic_max_nonneg(&bmax[s], mb);
  }
}

// Per system: relres, convergence mask, step count and status (a failure of
// the FP32 solve is passed on as it is); one block sets `done`.
__global__ __launch_bounds__(1024) void status_kernel(
    int64_t batch, double tol, unsigned long long* __restrict__ rmax,
    const unsigned long long* __restrict__ bmax, const int32_t* __restrict__ sinfo,
    int32_t* __restrict__ active, int32_t* __restrict__ steps, double* __restrict__ relres,
    int32_t* __restrict__ info, int32_t* __restrict__ done, int32_t step, int32_t last) {
  __shared__ int s_any;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  if (!*done) {
    for (int64_t s = threadIdx.x; s < batch; s += blockDim.x) {
      const double bn = as_double(bmax[s]);
      const double rn = as_double(rmax[s]);
      rmax[s] = 0ull;
      if (!active[s]) continue;
      const double rr = bn > 0.0 ? rn / bn : 0.0;
      relres[s] = rr;
      steps[s] = step + 1;
      if (sinfo[s] != 0) {  // FP32 solve: bad pivot or blocks that failed to meet
        active[s] = 0;
        info[s] = sinfo[s];
      } else if (!isfinite(rr)) {
        active[s] = 0;
        info[s] = -2;
      } else if (rr < tol) {
        active[s] = 0;
        info[s] = 0;
      } else if (last) {
        info[s] = -1;
      } else {
        s_any = 1;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && !*done && !s_any) *done = 1;
}

__global__ void init_flags_kernel(int64_t batch, int32_t* active, unsigned long long* rmax,
                                  unsigned long long* bmax, int32_t* steps, double* relres,
                                  int32_t* done) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < batch;
       s += (int64_t)gridDim.x * blockDim.x) {
    active[s] = 1;
    rmax[s] = 0ull;
    bmax[s] = 0ull;
    steps[s] = 0;
    relres[s] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *done = 0;
}

// The compact path is taken for the sweep's systems (a compact variant
// covers n and ld with FP64 storage) unless the FP32 state is off.
int compact_idx(int kind, int64_t n, int64_t ld) {
  return f32_compact_state() ? compact_pick(kind, 0, n, ld, 0) : -1;
}

struct Layout {
  int nplanes, cidx;
  int64_t plane;  // elements per plane
  size_t solver, a32, r32, r64, d32, act, sinfo, rmax, bmax, done, total;  // byte offsets
};

// The solver's workspace comes first, so its meeting counters sit at the
// same bytes on either path (a workspace may serve both in turn).
Layout layout(int kind, int64_t n, int64_t batch, int64_t ld) {
  Layout L;
  L.nplanes = kind == 5 ? 5 : 3;
  L.plane = n * ld;
  L.cidx = compact_idx(kind, n, ld);
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  size_t o = 0;
  L.solver = o;
  o = up(o + (L.cidx >= 0 ? compact_workspace_bytes(kind, L.cidx, n, batch)
                          : direct_ws_bytes(kind, 1, n, batch, ld)));
  L.a32 = L.r32 = L.r64 = L.d32 = o;
  if (L.cidx >= 0) {
    L.r64 = o;  o = up(o + (size_t)L.plane * 8);
  } else {
    L.a32 = o;  o = up(o + (size_t)L.nplanes * L.plane * 4);
    L.r32 = o;  o = up(o + (size_t)L.plane * 4);
    L.d32 = o;  o = up(o + (size_t)L.plane * 4);
  }
  L.act = o;  o = up(o + (size_t)batch * 4);
  L.sinfo = o; o = up(o + (size_t)batch * 4);
  L.rmax = o; o = up(o + (size_t)batch * 8);
  L.bmax = o; o = up(o + (size_t)batch * 8);
  L.done = o; o = up(o + 4);
  L.total = o;
  return L;
}

int grid_for(int64_t work) {
  const int64_t b = (work + kBlock - 1) / kBlock;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

}  // namespace

size_t refine_workspace_bytes(int kind, int64_t n, int64_t batch, int64_t ld) {
  return layout(kind, n, batch, ld).total;
}

hipError_t launch_refine(int kind, int64_t n, int64_t batch, int64_t ld, const double* const dg[5],
                         const double* rhs, double* x, double tol, int32_t max_steps,
                         int32_t* steps, double* relres, int32_t* info, void* ws,
                         hipStream_t st) {
  const Layout L = layout(kind, n, batch, ld);
  char* base = static_cast<char*>(ws);
  float* a32 = reinterpret_cast<float*>(base + L.a32);
  float* r32 = reinterpret_cast<float*>(base + L.r32);
  double* r64 = reinterpret_cast<double*>(base + L.r64);
  float* d32 = reinterpret_cast<float*>(base + L.d32);
  int32_t* act = reinterpret_cast<int32_t*>(base + L.act);
  int32_t* sinfo = reinterpret_cast<int32_t*>(base + L.sinfo);
  unsigned long long* rmax = reinterpret_cast<unsigned long long*>(base + L.rmax);
  unsigned long long* bmax = reinterpret_cast<unsigned long long*>(base + L.bmax);
  int32_t* done = reinterpret_cast<int32_t*>(base + L.done);
  double* sws = reinterpret_cast<double*>(base + L.solver);

  hipLaunchKernelGGL(init_flags_kernel, dim3(grid_for(batch)), dim3(kBlock), 0, st, batch, act,
                     rmax, bmax, steps, relres, done);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // rows of a system split over `parts` work items: about 2^19 items in all
  // (256 CUs x 32 waves x 64 lanes), at least one row each
  int64_t parts = ((int64_t(1) << 19) + batch - 1) / batch;
  if (parts > n) parts = n;
  const dim3 rgrid(grid_for(batch * parts));
  auto status = [&](int32_t step) {
    hipLaunchKernelGGL(status_kernel, dim3(1), dim3(1024), 0, st, batch, tol, rmax, bmax, sinfo,
                       act, steps, relres, info, done, step, (int32_t)(step == max_steps - 1));
    return hipGetLastError();
  };

  if (L.cidx >= 0) {
    // compact solves on the FP64 data: x = solve(b), then x += solve(r) for
    // the systems still refining
    for (int32_t step = 0; step < max_steps; ++step) {
      e = launch_compact_f64(kind, L.cidx, n, batch, ld, dg, step == 0 ? rhs : r64, x, sinfo, sws,
                             st, done, step > 0, step > 0 ? act : nullptr);
      if (e != hipSuccess) return e;
#define BS_RES(K, BN)                                                                              \
  hipLaunchKernelGGL((residual_kernel<K, double, BN>), rgrid, dim3(kBlock), 0, st, n, batch, ld,   \
                     dg[0], dg[1], dg[2], dg[3], dg[4], rhs, x, r64, rmax, parts, done, bmax, act)
      if (kind == 5) {
        if (step == 0) BS_RES(5, true); else BS_RES(5, false);
      } else {
        if (step == 0) BS_RES(3, true); else BS_RES(3, false);
      }
#undef BS_RES
      e = status(step);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  // FP32 storage: planes of A in the order of the FP32 copy (PD e c d a b, TD c d a)
  Planes pl;
  int np = 0;
  for (int k = 0; k < 5; ++k) pl.p[k] = nullptr;
  for (int k = 0; k < 5; ++k)
    if (kind == 5 || (k >= 1 && k <= 3)) pl.p[np++] = dg[k];
  hipLaunchKernelGGL(setup_kernel, dim3(grid_for(batch * parts)), dim3(kBlock), 0, st, n, batch,
                     ld, np, pl, a32, rhs, r32, x, bmax, parts);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const void* d32planes[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  {
    int q = 0;
    for (int k = 0; k < 5; ++k)
      if (kind == 5 || (k >= 1 && k <= 3)) d32planes[k] = a32 + (q++) * L.plane;
  }
  for (int32_t step = 0; step < max_steps; ++step) {
    e = launch_direct(kind, 1, n, batch, ld, d32planes, r32, d32, sinfo, sws, st, done);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(update_kernel, dim3(grid_for(n * batch)), dim3(kBlock), 0, st, n, batch,
                       ld, d32, x, act, done);
    if (kind == 5)
      hipLaunchKernelGGL((residual_kernel<5, float, false>), rgrid, dim3(kBlock), 0, st, n, batch,
                         ld, dg[0], dg[1], dg[2], dg[3], dg[4], rhs, x, r32, rmax, parts, done,
                         bmax, nullptr);
    else
      hipLaunchKernelGGL((residual_kernel<3, float, false>), rgrid, dim3(kBlock), 0, st, n, batch,
                         ld, dg[0], dg[1], dg[2], dg[3], dg[4], rhs, x, r32, rmax, parts, done,
                         bmax, nullptr);
    e = status(step);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace bs
