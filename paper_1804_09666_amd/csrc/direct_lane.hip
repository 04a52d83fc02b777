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
#include "seq_core.h"

#pragma clang fp contract(off)

namespace bs {
namespace {

constexpr int kLaneBlock = 64;  // one wave per block: spreads few systems over many CUs

__device__ inline bool bad_pivot(double m) { return !(m != 0.0) || !isfinite(m); }

constexpr int kPF = 8;  // rows in flight per lane (x <= 8 memory operations < 64)

// NPDM and NTDM (Thomas): the sequential sweeps of seq_core.h, one lane per
// system.  alpha (and beta) go through the workspace planes, z through x.
template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void direct_lane_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ E,
    const double* __restrict__ C, const double* __restrict__ D, const double* __restrict__ A,
    const double* __restrict__ B, const double* __restrict__ Y, double* __restrict__ X,
    int32_t* __restrict__ info, double* __restrict__ ws, int64_t lw) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch) return;
  auto fetch = [&](int64_t i) {
    const int64_t o = i * ld + s;
    seq::Row w;
    w.e = (KIND == 5) ? E[o] : 0.0;
    w.c = C[o];
    w.d = D[o];
    w.a = A[o];
    w.b = (KIND == 5) ? B[o] : 0.0;
    w.y = Y[o];
    return w;
  };
  const seq::Planes P{ws, ws + n * lw, lw, X, ld, s};
  const int64_t bad = seq::solve<KIND>(
      n, fetch, P, [&](int64_t i, double v) { X[i * ld + s] = v; },
      [](int64_t) { return true; });
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
// The carried state is (u0, u1, u2) of the two previous rows.
struct FactorState {
  double u0m1 = 0, u0m2 = 0, u1m1 = 0, u1m2 = 0, u2m1 = 0, u2m2 = 0;
};

// Row i of the recurrence with the rows before `lo` taken as absent (lo = 0:
// the recurrence itself; the corner slots e_0, e_1, c_0, a_{n-1}, b_{n-2},
// b_{n-1} are never used).  Returns u0 (the pivot) and advances the state.
template <int KIND>
__device__ inline void factor_row(int64_t i, int64_t lo, int64_t n, double e, double c, double d,
                                  double a, double b, FactorState& st, double& l2, double& l1,
                                  double& u0, double& u1) {
  const int64_t li = i - lo;
  double u2 = 0.0;
  l2 = 0.0;
  l1 = 0.0;
  u1 = 0.0;
  if (KIND == 5 && li >= 2) l2 = e / st.u0m2;
  if (li == 1) l1 = c / st.u0m1;
  if (li >= 2) l1 = (KIND == 5) ? (c - l2 * st.u1m2) / st.u0m1 : c / st.u0m1;
  if (li == 0)
    u0 = d;
  else if (li == 1 || KIND == 3)
    u0 = d - l1 * st.u1m1;
  else
    u0 = (d - l2 * st.u2m2) - l1 * st.u1m1;
  if (i <= n - 2) u1 = (li == 0 || KIND == 3) ? a : a - l1 * st.u2m1;
  if (KIND == 5 && i <= n - 3) u2 = b;
  st.u0m2 = st.u0m1; st.u0m1 = u0;
  st.u1m2 = st.u1m1; st.u1m1 = u1;
  st.u2m2 = st.u2m1; st.u2m1 = u2;
}

struct FactorPlanes {
  double* l2;  // KIND 5 only
  double* l1;
  double* u0;
  double* u1;  // KIND 5 only
};

template <int KIND>
__device__ inline FactorPlanes factor_planes(double* F, int64_t n, int64_t fld) {
  const int64_t plane = n * fld;
  if (KIND == 5) return {F, F + plane, F + 2 * plane, F + 3 * plane};
  return {nullptr, F, F + plane, nullptr};
}

// Rows [lo, hi) of system s, factors written for rows >= w0; returns the
// first row >= w0 whose pivot is zero or not finite (-1 if none).  The sweep
// runs on past a bad pivot (the later factors are unspecified).
template <int KIND>
__device__ inline int64_t factor_rows(int64_t n, int64_t ld, int64_t s, int64_t lo, int64_t w0,
                                      int64_t hi, const double* __restrict__ E,
                                      const double* __restrict__ C, const double* __restrict__ D,
                                      const double* __restrict__ A, const double* __restrict__ B,
                                      FactorPlanes P, int64_t fld) {
  double re[kPF], rc[kPF], rd[kPF], ra[kPF], rb[kPF];
  auto fetch = [&](int q, int64_t k) {
    const int64_t o = (lo + k) * ld + s;
    if (KIND == 5) re[q] = E[o];
    rc[q] = C[o];
    rd[q] = D[o];
    ra[q] = A[o];
    if (KIND == 5) rb[q] = B[o];
  };
  FactorState st;
  int64_t bad = -1;
  auto use = [&](int q, int64_t k) {
    const int64_t i = lo + k;
    double l2, l1, u0, u1;
    factor_row<KIND>(i, lo, n, KIND == 5 ? re[q] : 0.0, rc[q], rd[q], ra[q],
                     KIND == 5 ? rb[q] : 0.0, st, l2, l1, u0, u1);
    if (i >= w0) {
      if (bad < 0 && bad_pivot(u0)) bad = i;
      const int64_t fo = i * fld + s;
      if (KIND == 5) {
        P.l2[fo] = l2;
        P.u1[fo] = u1;
      }
      P.l1[fo] = l1;
      P.u0[fo] = u0;
    }
  };
  stream_rows<kPF, false>(hi - lo, fetch, use);
  return bad;
}

template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void factor_lane_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ E,
    const double* __restrict__ C, const double* __restrict__ D,
    const double* __restrict__ A, const double* __restrict__ B,
    double* __restrict__ F, int64_t fld, int32_t* __restrict__ info) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch) return;
  const int64_t bad = factor_rows<KIND>(n, ld, s, 0, 0, n, E, C, D, A, B,
                                        factor_planes<KIND>(F, n, fld), fld);
  info[s] = bad < 0 ? 0 : (int32_t)(bad + 1);
}

// ---- ILU(0) with the rows of a system split over lanes ------------------
// On the systems of the ADI sweeps the pivot recurrence forgets where it
// started: an error in the carried state shrinks by a factor of about
// c_i a_{i-1} / u0_{i-1}^2 < 1 per row.  So the rows of a system are cut into
// chunks of M rows; lane (s, k) starts kFactorWarm rows before its chunk as if
// the matrix began there, runs the recurrence through those warm-up rows
// (results dropped) and then through its own rows (written).  Once the state
// has converged to the bit, the chunk's factors are those of the sequential
// recurrence.  The proof kernel shows that it has: for every chunk it
// recomputes the chunk's first two rows from the stored factors of the two
// rows before it (the sequential state, by induction from chunk 0, which
// starts at row 0) and compares bit patterns; a system with any mismatch is
// factorized again, sequentially, by one lane of the finish kernel.  Either way the output is the
// sequential recurrence's to the last bit, and so is info.
// On the second-order sweeps at r = 4 the state reaches the sequential one
// to the bit within 57..64 rows (56 warm-up rows leave chunks unproven, 64
// do not); 80 leaves room for somewhat weaker dominance.  Where a system
// needs more, it is redone sequentially: the result is the same, only slower.
constexpr int64_t kFactorWarm = 80;
// lanes to aim for: the warm-up rows are read twice, so fewer, longer chunks
// win once the GPU has a few thousand waves of them (measured)
constexpr int64_t kFactorLanes[2] = {32768, 32768};  // PD, TD

__global__ void info_init_kernel(int64_t batch, int32_t* __restrict__ info) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < batch) info[s] = INT32_MAX;
}

template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void factor_chunk_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ E,
    const double* __restrict__ C, const double* __restrict__ D,
    const double* __restrict__ A, const double* __restrict__ B,
    double* __restrict__ F, int64_t fld, int32_t* __restrict__ info, int64_t M) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  const int64_t w0 = (int64_t)blockIdx.y * M;
  if (s >= batch) return;
  const int64_t lo = w0 > kFactorWarm ? w0 - kFactorWarm : 0;
  const int64_t hi = w0 + M < n ? w0 + M : n;
  const int64_t bad = factor_rows<KIND>(n, ld, s, lo, w0, hi, E, C, D, A, B,
                                        factor_planes<KIND>(F, n, fld), fld);
  if (bad >= 0) atomicMin(&info[s], (int32_t)(bad + 1));
}

__device__ inline bool same_bits(double a, double b) {
  return __double_as_longlong(a) == __double_as_longlong(b);
}

// One lane per (system, chunk boundary): recompute the chunk's first two
// rows from the stored rows before it and compare bit patterns; a mismatch
// marks the system (info < 0).
template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void factor_proof_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ E,
    const double* __restrict__ C, const double* __restrict__ D,
    const double* __restrict__ A, const double* __restrict__ B,
    const double* __restrict__ F, int64_t fld, int32_t* __restrict__ info, int64_t M) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch) return;
  // chunk k starts at row k M; those with k M <= kFactorWarm started at row 0
  const int64_t k = kFactorWarm / M + 1 + blockIdx.y;
  const int64_t r = k * M;  // kFactorWarm < r < n
  const FactorPlanes P = factor_planes<KIND>(const_cast<double*>(F), n, fld);
  FactorState st;
  for (int64_t i = r - 2; i < r; ++i) {  // the stored state of rows r-2, r-1
    const int64_t o = i * fld + s;
    st.u0m2 = st.u0m1;
    st.u1m2 = st.u1m1;
    st.u2m2 = st.u2m1;
    st.u0m1 = P.u0[o];
    st.u1m1 = (KIND == 5) ? P.u1[o] : (i <= n - 2 ? A[i * ld + s] : 0.0);
    st.u2m1 = (KIND == 5 && i <= n - 3) ? B[i * ld + s] : 0.0;
  }
  bool ok = true;
  for (int64_t i = r; i < r + 2 && i < n; ++i) {
    const int64_t o = i * ld + s, fo = i * fld + s;
    double l2, l1, u0, u1;
    factor_row<KIND>(i, 0, n, KIND == 5 ? E[o] : 0.0, C[o], D[o], A[o], KIND == 5 ? B[o] : 0.0,
                     st, l2, l1, u0, u1);
    ok = ok && same_bits(l1, P.l1[fo]) && same_bits(u0, P.u0[fo]);
    if (KIND == 5) ok = ok && same_bits(l2, P.l2[fo]) && same_bits(u1, P.u1[fo]);
  }
  if (!ok) atomicMin(&info[s], -1);
}

// One lane per system: proven systems report the first bad pivot the chunk
// lanes saw (their rows are the sequential ones); the others are factorized
// again, sequentially.
template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void factor_finish_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ E,
    const double* __restrict__ C, const double* __restrict__ D,
    const double* __restrict__ A, const double* __restrict__ B,
    double* __restrict__ F, int64_t fld, int32_t* __restrict__ info) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch) return;
  const int32_t b = info[s];
  if (b >= 0) {
    info[s] = b == INT32_MAX ? 0 : b;
    return;
  }
  const int64_t bad = factor_rows<KIND>(n, ld, s, 0, 0, n, E, C, D, A, B,
                                        factor_planes<KIND>(F, n, fld), fld);
  info[s] = bad < 0 ? 0 : (int32_t)(bad + 1);
}

// Substitution with the band factors: z_i = (y_i - l1_i z_{i-1}) - l2_i z_{i-2},
// then x_i = ((z_i - u1_i x_{i+1}) - u2_i x_{i+2}) / u0_i.
// Row i of the factor planes sits at i * fld, of A's arrays at i * ald.
struct SubstPlanes {
  const double* l2;  // KIND 5 only
  const double* l1;
  const double* u0;
  const double* u1;  // KIND 5: the u1 plane (pitch fld); KIND 3: a (pitch ald)
  const double* u2;  // KIND 5: b (pitch ald)
  int64_t fld, ald;
};

template <int KIND>
__host__ __device__ inline SubstPlanes subst_planes(const double* F, int64_t fld, const double* Aa,
                                           const double* B, int64_t n, int64_t ald) {
  const int64_t plane = n * fld;
  if (KIND == 5) return {F, F + plane, F + 2 * plane, F + 3 * plane, B, fld, ald};
  return {nullptr, F, F + plane, Aa, nullptr, fld, ald};
}

// Vectors of one substitution: rhs y (pitch yl), z (pitch zl), x (pitch xl);
// `active` (nullable): systems with active[s] == 0 are left alone; `done`
// (nullable): the whole launch returns at once when *done != 0.
struct SubstIO {
  const double* y;
  int64_t yl;
  double* z;
  int64_t zl;
  double* x;
  int64_t xl;
  const int32_t* active;
  const int32_t* done;
};

__device__ inline bool subst_idle(const SubstIO& io, int64_t s) {
  return (io.done != nullptr && *io.done) || (io.active != nullptr && io.active[s] == 0);
}

// Forward rows [lo, hi) of system s with z_{lo-1}, z_{lo-2} taken as absent;
// z written for rows >= w0.
template <int KIND>
__device__ inline void subst_fwd_rows(int64_t s, int64_t lo, int64_t w0, int64_t hi,
                                      SubstPlanes P, const SubstIO& io) {
  double ry[kPF], rl1[kPF], rl2[kPF];
  double zm1 = 0, zm2 = 0;
  auto fetch = [&](int q, int64_t k) {
    const int64_t i = lo + k, fo = i * P.fld + s;
    ry[q] = io.y[i * io.yl + s];
    rl1[q] = P.l1[fo];
    if (KIND == 5) rl2[q] = P.l2[fo];
  };
  auto use = [&](int q, int64_t k) {
    double t = ry[q];
    if (k >= 1) t = t - rl1[q] * zm1;
    if (KIND == 5 && k >= 2) t = t - rl2[q] * zm2;
    if (lo + k >= w0) io.z[(lo + k) * io.zl + s] = t;
    zm2 = zm1;
    zm1 = t;
  };
  stream_rows<kPF, false>(hi - lo, fetch, use);
}

// Backward rows top-1 down to w0 of system s with x_top, x_{top+1} taken as
// absent (top = n: the recurrence itself); x written for rows < w1.
template <int KIND>
__device__ inline void subst_bwd_rows(int64_t s, int64_t w0, int64_t w1, int64_t top,
                                      SubstPlanes P, const SubstIO& io) {
  double rz[kPF], ru1[kPF], ru2[kPF], ru0[kPF];
  double xp1 = 0, xp2 = 0;
  const int64_t u1l = KIND == 5 ? P.fld : P.ald;
  auto fetch = [&](int q, int64_t k) {
    const int64_t i = w0 + k;
    rz[q] = io.z[i * io.zl + s];
    ru1[q] = P.u1[i * u1l + s];
    if (KIND == 5) ru2[q] = P.u2[i * P.ald + s];
    ru0[q] = P.u0[i * P.fld + s];
  };
  auto use = [&](int q, int64_t k) {
    const int64_t i = w0 + k;
    double t = rz[q];
    if (i + 1 < top) t = t - ru1[q] * xp1;
    if (KIND == 5 && i + 2 < top) t = t - ru2[q] * xp2;
    const double xi = t / ru0[q];
    if (i < w1) io.x[i * io.xl + s] = xi;
    xp2 = xp1;
    xp1 = xi;
  };
  stream_rows<kPF, true>(top - w0, fetch, use);
}

template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void subst_lane_kernel(
    int64_t n, int64_t batch, int64_t ld, const double* __restrict__ Aa,
    const double* __restrict__ B, const double* __restrict__ F, int64_t fld,
    const double* __restrict__ Y, double* __restrict__ X, int32_t* __restrict__ info) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch) return;
  const SubstPlanes P = subst_planes<KIND>(F, fld, Aa, B, n, ld);
  const SubstIO io{Y, ld, X, ld, X, ld, nullptr, nullptr};  // z kept in x
  subst_fwd_rows<KIND>(s, 0, 0, n, P, io);
  subst_bwd_rows<KIND>(s, 0, n, n, P, io);
  info[s] = 0;
}

// ---- substitution with the rows of a system split over lanes ------------
// Both sweeps are linear recurrences whose homogeneous parts shrink an error
// in the carried pair by about |l1| (forward) and |u1 / u0| (backward) per
// row, so they are cut into chunks exactly like the factorization: each lane
// starts kSubstWarm rows early (forward: before its chunk; backward: after
// it) with the pair outside taken as absent, and a proof kernel recomputes the
// two rows at every chunk boundary from the stored rows beyond it; a fix
// kernel redoes the sweep of a system sequentially where any bit differs.
// z goes through the workspace ([n][ws_ld] doubles, then the flags), so the
// backward warm-up never reads a row another lane has already overwritten
// with x.
// at r = 4 the sweeps need 113..128 rows (|l1| and |u1/u0| reach ~0.7)
constexpr int64_t kSubstWarm = 128;
constexpr int64_t kSubstLanes = 32768;

// flags[s] (int32, workspace) marks a system whose proof failed; the forward
// chunk kernel clears it, each fix kernel acts on it and clears it again.
template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void subst_fwd_chunk_kernel(
    int64_t n, int64_t batch, SubstPlanes P, SubstIO io, int32_t* __restrict__ flags, int64_t M) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch || subst_idle(io, s)) return;
  if (blockIdx.y == 0) flags[s] = 0;
  const int64_t w0 = (int64_t)blockIdx.y * M;
  const int64_t lo = w0 > kSubstWarm ? w0 - kSubstWarm : 0;
  const int64_t hi = w0 + M < n ? w0 + M : n;
  subst_fwd_rows<KIND>(s, lo, w0, hi, P, io);
}

// One lane per (system, chunk that started early): z of the chunk's first
// two rows from the stored z of the two rows before it.
template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void subst_fwd_proof_kernel(
    int64_t n, int64_t batch, SubstPlanes P, SubstIO io, int32_t* __restrict__ flags, int64_t M) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch || subst_idle(io, s)) return;
  const int64_t r = (kSubstWarm / M + 1 + blockIdx.y) * M;  // kSubstWarm < r < n
  double zm2 = io.z[(r - 2) * io.zl + s], zm1 = io.z[(r - 1) * io.zl + s];
  bool ok = true;
  for (int64_t i = r; i < r + 2 && i < n; ++i) {
    const int64_t fo = i * P.fld + s;
    double t = io.y[i * io.yl + s];
    t = t - P.l1[fo] * zm1;
    if (KIND == 5) t = t - P.l2[fo] * zm2;
    ok = ok && same_bits(t, io.z[i * io.zl + s]);
    zm2 = zm1;
    zm1 = t;
  }
  if (!ok) flags[s] = 1;
}

template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void subst_fwd_fix_kernel(
    int64_t n, int64_t batch, SubstPlanes P, SubstIO io, int32_t* __restrict__ flags) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch || subst_idle(io, s) || flags[s] == 0) return;
  subst_fwd_rows<KIND>(s, 0, 0, n, P, io);
  flags[s] = 0;
}

template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void subst_bwd_chunk_kernel(
    int64_t n, int64_t batch, SubstPlanes P, SubstIO io, int64_t M) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch || subst_idle(io, s)) return;
  const int64_t w0 = (int64_t)blockIdx.y * M;
  const int64_t w1 = w0 + M < n ? w0 + M : n;
  const int64_t top = n - w1 > kSubstWarm ? w1 + kSubstWarm : n;
  subst_bwd_rows<KIND>(s, w0, w1, top, P, io);
}

// One lane per (system, chunk that started late): x of the chunk's last two
// rows from the stored x of the two rows after it.  Chunk k ends at row
// (k + 1) M; those within kSubstWarm rows of n ran from n.
template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void subst_bwd_proof_kernel(
    int64_t n, int64_t batch, SubstPlanes P, SubstIO io, int32_t* __restrict__ flags, int64_t M) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch || subst_idle(io, s)) return;
  const int64_t w1 = ((int64_t)blockIdx.y + 1) * M;  // n - w1 > kSubstWarm
  const int64_t u1l = KIND == 5 ? P.fld : P.ald;
  double xp1 = io.x[w1 * io.xl + s], xp2 = io.x[(w1 + 1) * io.xl + s];
  bool ok = true;
  for (int64_t i = w1 - 1; i >= w1 - 2; --i) {
    double t = io.z[i * io.zl + s];
    t = t - P.u1[i * u1l + s] * xp1;
    if (KIND == 5) t = t - P.u2[i * P.ald + s] * xp2;
    const double xi = t / P.u0[i * P.fld + s];
    ok = ok && same_bits(xi, io.x[i * io.xl + s]);
    xp2 = xp1;
    xp1 = xi;
  }
  if (!ok) flags[s] = 1;
}

template <int KIND>
__global__ __launch_bounds__(kLaneBlock) void subst_bwd_fix_kernel(
    int64_t n, int64_t batch, SubstPlanes P, SubstIO io, int32_t* __restrict__ info,
    int32_t* __restrict__ flags) {
  const int64_t s = (int64_t)blockIdx.x * kLaneBlock + threadIdx.x;
  if (s >= batch || subst_idle(io, s)) return;
  if (flags[s] != 0) {
    subst_bwd_rows<KIND>(s, 0, n, n, P, io);
    flags[s] = 0;
  }
  if (info != nullptr) info[s] = 0;
}

inline dim3 lane_grid(int64_t batch) {
  return dim3((unsigned)((batch + kLaneBlock - 1) / kLaneBlock));
}

}  // namespace

hipError_t launch_npdm_lane(int64_t n, int64_t batch, int64_t ld, Diags A,
                            const double* y, double* x, int32_t* info,
                            double* ws, hipStream_t st) {
  hipLaunchKernelGGL(direct_lane_kernel<5>, lane_grid(batch),
                     dim3(kLaneBlock), 0, st, n, batch, ld, A.e, A.c, A.d, A.a,
                     A.b, y, x, info, ws, ws_ld(batch));
  return hipGetLastError();
}

hipError_t launch_ntdm_lane(int64_t n, int64_t batch, int64_t ld, Diags A,
                            const double* y, double* x, int32_t* info,
                            double* ws, hipStream_t st) {
  hipLaunchKernelGGL(direct_lane_kernel<3>, lane_grid(batch),
                     dim3(kLaneBlock), 0, st, n, batch, ld, nullptr, A.c, A.d, A.a,
                     nullptr, y, x, info, ws, ws_ld(batch));
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

hipError_t launch_factor(int kind, int64_t n, int64_t batch, int64_t ld, Diags A,
                         double* factors, int64_t fld, int32_t* info, hipStream_t st) {
  // chunks of at least 64 rows, enough of them for about `lanes` lanes
  const int64_t lanes = kFactorLanes[kind == 5 ? 0 : 1];
  int64_t K = (lanes + batch - 1) / batch;
  if (K > n / 64) K = n / 64;
  if (K > 4096) K = 4096;  // grid y limit; far more lanes than the GPU holds
  if (K <= 1) return launch_factor_lane(kind, n, batch, ld, A, factors, fld, info, st);
  const int64_t M = (n + K - 1) / K;
  K = (n + M - 1) / M;
  hipLaunchKernelGGL(info_init_kernel, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, st,
                     batch, info);
  const unsigned gx = (unsigned)((batch + kLaneBlock - 1) / kLaneBlock);
  const int64_t proofs = K - (kFactorWarm / M + 1);  // chunks that started early
  if (kind == 5) {
    hipLaunchKernelGGL(factor_chunk_kernel<5>, dim3(gx, (unsigned)K), dim3(kLaneBlock), 0, st, n,
                       batch, ld, A.e, A.c, A.d, A.a, A.b, factors, fld, info, M);
    if (proofs > 0)
      hipLaunchKernelGGL(factor_proof_kernel<5>, dim3(gx, (unsigned)proofs), dim3(kLaneBlock), 0,
                         st, n, batch, ld, A.e, A.c, A.d, A.a, A.b, factors, fld, info, M);
    hipLaunchKernelGGL(factor_finish_kernel<5>, dim3(gx), dim3(kLaneBlock), 0, st, n, batch, ld,
                       A.e, A.c, A.d, A.a, A.b, factors, fld, info);
  } else {
    hipLaunchKernelGGL(factor_chunk_kernel<3>, dim3(gx, (unsigned)K), dim3(kLaneBlock), 0, st, n,
                       batch, ld, A.e, A.c, A.d, A.a, A.b, factors, fld, info, M);
    if (proofs > 0)
      hipLaunchKernelGGL(factor_proof_kernel<3>, dim3(gx, (unsigned)proofs), dim3(kLaneBlock), 0,
                         st, n, batch, ld, A.e, A.c, A.d, A.a, A.b, factors, fld, info, M);
    hipLaunchKernelGGL(factor_finish_kernel<3>, dim3(gx), dim3(kLaneBlock), 0, st, n, batch, ld,
                       A.e, A.c, A.d, A.a, A.b, factors, fld, info);
  }
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

int64_t subst_chunks(int64_t n, int64_t batch) {
  int64_t K = (kSubstLanes + batch - 1) / batch;
  if (K > n / 128) K = n / 128;  // chunks of at least 128 rows
  if (K > 4096) K = 4096;
  return K < 1 ? 1 : K;
}

size_t subst_workspace_bytes(int64_t n, int64_t batch) {
  if (subst_chunks(n, batch) <= 1) return 0;
  return (size_t)(n * ws_ld(batch)) * 8 + (size_t)(batch * 4 + 255) / 256 * 256;
}

// The split substitution of systems with active != 0 (all when NULL): y
// (pitch yl) -> x (pitch ld), factors of pitch fld; z and the flags in ws;
// every launch returns at once when done != NULL and *done != 0.
hipError_t launch_subst_masked(int kind, int64_t n, int64_t batch, int64_t ld, Diags A,
                               const double* factors, int64_t fld, const double* y, int64_t yl,
                               double* x, int32_t* info, double* ws, const int32_t* active,
                               const int32_t* done, hipStream_t st) {
  int64_t K = subst_chunks(n, batch);
  if (K <= 1) return hipErrorInvalidValue;
  const int64_t M = (n + K - 1) / K;
  K = (n + M - 1) / M;
  const int64_t zl = ws_ld(batch);
  int32_t* flags = reinterpret_cast<int32_t*>(ws + n * zl);
  const unsigned gx = (unsigned)((batch + kLaneBlock - 1) / kLaneBlock);
  const dim3 grid(gx, (unsigned)K), lanes(kLaneBlock);
  const SubstIO io{y, yl, ws, zl, x, ld, active, done};
  // forward proofs: chunks that started before row 0 of their own (k M > warm-up)
  const int64_t fproofs = K - (kSubstWarm / M + 1);
  // backward proofs: chunks whose end lies more than the warm-up before n
  int64_t bproofs = 0;
  while (bproofs < K - 1 && n - (bproofs + 1) * M > kSubstWarm) ++bproofs;
#define BS_SUBST(KD)                                                                          \
  {                                                                                           \
    const SubstPlanes P = subst_planes<KD>(factors, fld, A.a, A.b, n, ld);                    \
    hipLaunchKernelGGL(subst_fwd_chunk_kernel<KD>, grid, lanes, 0, st, n, batch, P, io,       \
                       flags, M);                                                             \
    if (fproofs > 0)                                                                          \
      hipLaunchKernelGGL(subst_fwd_proof_kernel<KD>, dim3(gx, (unsigned)fproofs), lanes, 0,   \
                         st, n, batch, P, io, flags, M);                                      \
    hipLaunchKernelGGL(subst_fwd_fix_kernel<KD>, dim3(gx), lanes, 0, st, n, batch, P, io,     \
                       flags);                                                                \
    hipLaunchKernelGGL(subst_bwd_chunk_kernel<KD>, grid, lanes, 0, st, n, batch, P, io, M);   \
    if (bproofs > 0)                                                                          \
      hipLaunchKernelGGL(subst_bwd_proof_kernel<KD>, dim3(gx, (unsigned)bproofs), lanes, 0,   \
                         st, n, batch, P, io, flags, M);                                      \
    hipLaunchKernelGGL(subst_bwd_fix_kernel<KD>, dim3(gx), lanes, 0, st, n, batch, P, io,     \
                       info, flags);                                                          \
  }
  if (kind == 5) {
    BS_SUBST(5)
  } else {
    BS_SUBST(3)
  }
#undef BS_SUBST
  return hipGetLastError();
}

hipError_t launch_subst(int kind, int64_t n, int64_t batch, int64_t ld, Diags A,
                        const double* factors, const double* y, double* x, int32_t* info,
                        double* ws, hipStream_t st) {
  if (subst_chunks(n, batch) <= 1)
    return launch_subst_lane(kind, n, batch, ld, A, factors, y, x, info, st);
  return launch_subst_masked(kind, n, batch, ld, A, factors, ld, y, ld, x, info, ws, nullptr,
                             nullptr, st);
}

hipError_t launch_subst_lane(int kind, int64_t n, int64_t batch, int64_t ld,
                             Diags A, const double* factors, const double* y,
                             double* x, int32_t* info, hipStream_t st) {
  if (kind == 5)
    hipLaunchKernelGGL(subst_lane_kernel<5>, lane_grid(batch),
                       dim3(kLaneBlock), 0, st, n, batch, ld, A.a, A.b,
                       factors, ld, y, x, info);
  else
    hipLaunchKernelGGL(subst_lane_kernel<3>, lane_grid(batch),
                       dim3(kLaneBlock), 0, st, n, batch, ld, A.a, A.b,
                       factors, ld, y, x, info);
  return hipGetLastError();
}

}  // namespace bs
