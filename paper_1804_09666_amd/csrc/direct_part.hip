// direct_part.hip -- NPDM / NTDM with the rows of each system split over many
// lanes, for batches too small to fill the GPU with one lane per system.
//
// Method (partitioned elimination).  System s is cut into P chunks of M rows;
// lane (s, j) owns chunk j.  Rows past n are identity rows, which leave the
// solution of the real rows unchanged.
//   1. The lane loads its M rows of e, c, d, a, b, y into registers (one
//      coalesced segment per row and group of G systems) and runs the NPDM
//      recurrences (the LU of Sec. 1 of Veneva & Ayriyan, arXiv:1804.09666)
//      on its chunk alone.  The couplings to the two rows before the chunk
//      (x_L) and the two rows after it (x_R) are carried as extra right-hand
//      sides, so after the back substitution every row of the chunk reads
//          x_r = p_r - V_r x_L - W_r x_R.
//      Rows 0, 1 and M-2, M-1 of (p, V, W) form the chunk's affine map from
//      (x_L, x_R) to its top pair T and bottom pair B.
//   2. Neighbouring maps are merged pairwise up a binary tree in LDS: merging
//      eliminates the interface pair (bottom of the left part, top of the
//      right part) with one NB x NB solve, and the node keeps the
//      affine expressions of that interface in terms of the outer x_L, x_R.
//      The root has no outer couplings (x_L = x_R = 0 at the system ends);
//      walking back down the tree hands every chunk its own x_L, x_R.
//   3. Each lane writes x_r = p_r - V_r x_L - W_r x_R for its rows.
// Inputs are read once and x written once: nothing goes through global
// scratch.  NB = 2 for pentadiagonal, 1 for tridiagonal systems.
//
// Block -> system-group mapping is XCD-aware: consecutive system groups
// (which share 128-byte lines of every row) go to the same XCD, so the line
// is fetched from HBM once and served from that XCD's L2 to its neighbours.
#include <algorithm>
#include <atomic>

#include "seq_core.h"
#include "split_core.h"

namespace bs {
namespace {

using namespace split;

// One block = G systems x PW chunks of M rows = one tile of RT = M*PW rows of
// G systems.  T <= TMAX tiles (consecutive blocks on one XCD) cover a system;
// they exchange their tile maps through `xch` and meet at the four counters
// cnt[4*grp ..] (arrivals, departures, mask of tiles that gave up waiting,
// mask of systems to redo; reset by the last tile to leave, so they are zero
// again after every completed call).  A tile waits at most wait_ticks of the
// 100 MHz real-time clock for the others, then gives up.
//
// Breakdown.  A system whose partitioned elimination meets a pivot or an
// interface block that the guard rejects (zero, tiny or not finite) is
// solved again with the sequential recurrence (seq_core.h), by one lane of
// the last tile of its group to leave (the only tile when T = 1), so its x
// and info are the sequential method's.  Every tile that read all tile maps
// reaches the same verdict and writes no x for such a system.  A tile that
// gave up writes no x at all; the last tile then solves the rows of the
// tiles that gave up sequentially (unless x aliases the rhs, whose rows the
// other tiles have overwritten: info = -4, x unspecified).  The sequential
// sweeps keep alpha, beta and z in the planes at rws (pitch rpitch).
// SPARSE: the outer diagonals come from an MNPDM list (absent entries are
// zero, so every product with them is an exact zero).
// ASM: the rows are assembled from the sweep input v (passed as Y) and r
// instead of being loaded (the ADI sweep of the PDE, see assemble_chunk).
// TS: type of the per-row chunk state: double, or float for the compact
// state of FP32 storage (chunk_pd_rows / chunk_td_rows on float arrays).
// ACC (compact state, FP64 x only): x += the solution instead of x = (a
// refinement step's correction).
constexpr int kListScan = 8;  // MNPDM lists up to this length: scanned by every lane
constexpr int kListLds = 64;  // longer ones up to this length: staged in LDS

template <typename TIO, int KIND, int M, int PW, int G, int TMAX, int WPE, bool SPARSE = false,
          bool ASM = false, typename TS = double, bool ACC = false>
__global__ __launch_bounds__(G * PW) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void part_kernel(
    int64_t n, int64_t batch, int64_t ld, const TIO* __restrict__ E,
    const TIO* __restrict__ C, const TIO* __restrict__ D,
    const TIO* __restrict__ A, const TIO* __restrict__ B,
    const TIO* __restrict__ Y, TIO* __restrict__ X,
    int32_t* __restrict__ info, double* __restrict__ xch,
    unsigned* __restrict__ cnt, int T, const int32_t* __restrict__ skip, Outer ol,
    double rcoef, uint64_t wait_ticks, double* __restrict__ rws, int64_t rpitch, int redo_gaveup,
    const int32_t* __restrict__ act) {
  constexpr int NB = KIND == 5 ? 2 : 1;
  constexpr int RS = kRecSz<NB>;
  constexpr int RT = M * PW;
  static_assert((PW & (PW - 1)) == 0 && (TMAX & (TMAX - 1)) == 0 && M >= 4, "shape");
  static_assert(G <= 32 && TMAX <= 32, "masks");
  static_assert(G >= 16, "the counter region is sized for groups of at least 16 systems");
  static_assert(sizeof(TS) == 8 || (!ASM && !SPARSE), "compact state");
  static_assert(!ACC || (sizeof(TS) == 4 && sizeof(TIO) == 8), "accumulating store");
  if (skip != nullptr && *skip) return;  // uniform: a refinement loop has finished
  __shared__ double s_node[(PW - 1) * G * RS];
  __shared__ double s_gnode[(TMAX > 1 ? TMAX - 1 : 1) * G * RS];
  __shared__ double s_bnd[G * 2 * NB];
  __shared__ int s_bad[G];
  __shared__ int s_timeout;
  // MNPDM: the block's lists in LDS (entry k of system g at [k * G + g]), up
  // to kListLds entries per system; their used lengths and verdicts
  __shared__ int32_t s_lrow[SPARSE ? kListLds * G : 1];
  __shared__ double s_le[SPARSE ? kListLds * G : 1], s_lb[SPARSE ? kListLds * G : 1];
  __shared__ int s_lcnt[SPARSE ? G : 1], s_lbad[SPARSE ? G : 1];

  const int tid = threadIdx.x;
  const int g = tid % G;
  const int j = tid / G;
  // block -> (system group, tile); the T tiles of a group sit on one XCD
  int64_t grp, tile;
  {
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
  const int64_t s = grp * G + g;
  // act (nullable): systems with act[s] == 0 are left alone (no loads, no
  // stores, no info)
  const bool live = s < batch && (act == nullptr || act[s] != 0);
  const int64_t r0 = (tile * PW + j) * M;
  if (tid < G) s_bad[tid] = kBadNone;
  if (tid == 0) s_timeout = 0;

  // ---- 1. load the chunk and eliminate it locally -------------------------
  TS p[M], v[NB][M], w[NB][M];
  int bad;
  bool list_bad = false;
  // rows in flight: at most 63 loads per wave; at two waves per SIMD the
  // register budget halves
  // (compact state: 8 rows of FP32 loads measured best, 43.6 against 44.7 us
  // for 10 on the PD sweep batch; 6 rows of FP64 loads keep its registers)
  constexpr int DPF = sizeof(TS) == 4 ? (sizeof(TIO) == 4 ? 8 : 6)
                      : WPE == 1 ? (KIND == 5 && !SPARSE ? 10 : 15) : (KIND == 5 ? 6 : 9);
  if constexpr (ASM) {
    stream_assemble<KIND, M>(n, ld, s, live, r0, reinterpret_cast<const double*>(Y), rcoef, p,
                             v, w, bad);
  } else {
    double eo[M], bo[M];
#pragma unroll
    for (int r = 0; r < M; ++r) eo[r] = bo[r] = 0.0;
    if constexpr (SPARSE) {
      // A list is valid when its used entries (row >= 0) come first, in
      // strictly ascending rows in [0, n).  Lists of kListScan entries or
      // fewer per system, and lists longer than kListLds, are scanned in
      // global memory by every lane (a few loads, no barrier: 61.9 against
      // 64.6 us with the LDS path at K = 2 on the sweep batch); in between,
      // the block stages its systems' lists in LDS once (loads of consecutive
      // systems), one lane per system checks its list there, and every lane
      // finds its rows by binary search.
      auto pick = [&](int32_t rr, double ev, double bv) __attribute__((always_inline)) {
        const int64_t loc = rr - r0;
        ev = (rr >= 2) ? ev : 0.0;
        bv = (rr <= n - 3) ? bv : 0.0;
        // a select per register (an indexed store would put eo, bo in memory)
#pragma unroll
        for (int r = 0; r < M; ++r) {
          eo[r] = (loc == r) ? ev : eo[r];
          bo[r] = (loc == r) ? bv : bo[r];
        }
      };
      if (ol.kmax > kListScan && ol.kmax <= kListLds) {  // uniform
        for (int q = tid; q < ol.kmax * G; q += G * PW) {
          const int k = q / G, gg = q % G;
          const int64_t sg = grp * G + gg;
          const bool lv = sg < batch && (act == nullptr || act[sg] != 0);
          const int64_t lo = (int64_t)k * ld + sg;
          s_lrow[q] = lv ? ol.row[lo] : -1;
          s_le[q] = lv ? ol.e[lo] : 0.0;
          s_lb[q] = lv ? ol.b[lo] : 0.0;
        }
        __syncthreads();
        if (j == 0) {
          int64_t prev = -1;
          int cnt = 0;
          bool ended = false, lbad = false;
          for (int k = 0; k < ol.kmax; ++k) {
            const int32_t rr = s_lrow[k * G + g];
            if (rr < 0) {
              ended = true;
            } else if (ended || rr >= n || rr <= prev) {
              lbad = true;
            } else {
              prev = rr;
              cnt = k + 1;
            }
          }
          s_lcnt[g] = cnt;
          s_lbad[g] = lbad;
        }
        __syncthreads();
        list_bad = live && s_lbad[g] != 0;
        if (live && !list_bad) {
          int lo = 0, hi = s_lcnt[g];  // first entry with row >= r0
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_lrow[mid * G + g] < r0)
              lo = mid + 1;
            else
              hi = mid;
          }
          for (int k = lo; k < s_lcnt[g] && s_lrow[k * G + g] < r0 + M; ++k)
            pick(s_lrow[k * G + g], s_le[k * G + g], s_lb[k * G + g]);
        }
      } else {
        int64_t prev = -1;
        bool ended = false;
        for (int k = 0; k < ol.kmax; ++k) {
          const int64_t lo = (int64_t)k * ld + s;
          const int32_t rr = live ? ol.row[lo] : -1;
          if (rr < 0) {
            ended = true;
            continue;
          }
          if (ended || rr >= n || rr <= prev) {
            list_bad = true;
            continue;
          }
          prev = rr;
          const int64_t loc = rr - r0;
          if (loc >= 0 && loc < M) {
            const double ev = (rr >= 2) ? ol.e[lo] : 0.0;
            const double bv = (rr <= n - 3) ? ol.b[lo] : 0.0;
#pragma unroll
            for (int r = 0; r < M; ++r)
              if (loc == r) {
                eo[r] = ev;
                bo[r] = bv;
              }
          }
        }
      }
    }
    // loads streamed under the forward elimination
    stream_eliminate<KIND, M, DPF, TIO, SPARSE, TS>(n, ld, s, live, r0, E, C, D, A, B, Y, eo, bo,
                                                    p, v, w, bad);
  }
  Map<NB> mp = chunk_map<NB, M>(p, v, w);
  __syncthreads();  // s_bad initialised
  if (bad < M && r0 + bad < n) atomicMin(&s_bad[g], (int)(r0 + bad + 1));

  // ---- 2. merge the chunks of this tile ----------------------------------
  tree_up<NB, PW, G>(mp, j, g, s_node, s_bad, M, tile * RT, n);

  double xl[NB], xr[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) xl[q] = xr[q] = 0.0;  // no coupling at the ends
  if (T > 1) {
    // ---- 2b. exchange tile maps with the other tiles of the system ------
    // The maps go through the device-coherent level with write-through
    // stores and cache-bypassing loads, so no cache-wide write-back or
    // invalidate is needed; the arrival count is bumped only after this
    // wave's map stores have been acknowledged (s_waitcnt), and a tile reads
    // the maps only after its own load of the counter has returned T.
    constexpr int XS = RS + 1;  // map + first bad row of the tile
    if (tid < 64) {  // wave 0 holds the tile maps (lanes j == 0, tid < G)
      if (j == 0) {
        double* dst = xch + ((grp * T + tile) * G + g) * XS;
        const double* src = reinterpret_cast<const double*>(&mp);
#pragma unroll
        for (int q = 0; q < RS; ++q) st_coherent(dst + q, src[q]);
        st_coherent(dst + RS, (double)s_bad[g]);
      }
      __builtin_amdgcn_s_waitcnt(kWaitVmem);
      if (tid == 0) {
        // the last tile to arrive has nothing to wait for
        if (atomicAdd(&cnt[4 * grp], 1u) + 1 < (unsigned)T) {
          const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
          while (ld_counter(&cnt[4 * grp]) < (unsigned)T) {
            __builtin_amdgcn_s_sleep(2);
            if (__builtin_amdgcn_s_memrealtime() - t0 > wait_ticks) {
              s_timeout = 1;
              break;
            }
          }
        }
      }
    }
    __syncthreads();
    Map<NB> gm;
    if (j < TMAX) {
      if (j < T) {
        const double* src = xch + ((grp * T + j) * G + g) * XS;
        double* dst = reinterpret_cast<double*>(&gm);
#pragma unroll
        for (int q = 0; q < RS; ++q) dst[q] = ld_coherent(src + q);
        const double tb = ld_coherent(src + RS);
        if (tb < (double)kBadNone) atomicMin(&s_bad[g], (int)tb);
      } else {  // tiles past the last one: all identity rows
        zero_map(gm);
      }
    }
    __syncthreads();  // every tile map read: this tile may leave (at the end)
    if constexpr (TMAX > 1) {
      tree_up<NB, TMAX, G>(gm, j, g, s_gnode, s_bad, RT, 0, n);
      double gl[NB], gr[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) gl[q] = gr[q] = 0.0;
      __syncthreads();
      tree_down<NB, TMAX, G>(gl, gr, j, g, s_gnode);
      if (j == tile) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          s_bnd[g * 2 * NB + q] = gl[q];
          s_bnd[g * 2 * NB + NB + q] = gr[q];
        }
      }
      __syncthreads();
      if (j == 0) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          xl[q] = s_bnd[g * 2 * NB + q];
          xr[q] = s_bnd[g * 2 * NB + NB + q];
        }
      }
    }
  }
  __syncthreads();
  // s_bad and s_timeout are final: read them before the walk down, which
  // hides the LDS latency
  const bool redo = s_bad[g] != kBadNone && !list_bad;
  const bool write = live && !s_timeout && !redo;

  // ---- 3. back down the tile's tree, then x = p - V x_L - W x_R ---------
  tree_down<NB, PW, G>(xl, xr, j, g, s_node);
  if constexpr (sizeof(TS) == 4)
    write_chunk<NB, M, TIO, ACC>(n, ld, s, write, r0, 0, p, v, w, xl, xr, X);
  else
    write_chunk<NB, M>(n, ld, s, write, r0, 0, p, v, w, xl, xr, X);
  // info at the device-coherent level: the last tile to leave may overwrite
  // it from another XCD
  if (j == 0 && tile == 0 && live && !s_timeout && !redo)
    st_coherent_i32(&info[s], list_bad ? kBadList : 0);

  // ---- 4. the sequential redo --------------------------------------------
  // Lane g of the redoing tile solves system g; rows i with keep(i) are
  // written (all rows, or the rows of the tiles that gave up).
  auto redo_system = [&](uint32_t tiles_mask) {
    int kc = 0;  // cursor in the staged list (MNPDM)
    auto fetch = [&](int64_t i) {
      const int64_t o = i * ld + s;
      seq::Row rw;
      if constexpr (ASM) {
        const double* V = reinterpret_cast<const double*>(Y);
        const double vm = (i >= 1) ? V[o - ld] : 0.0;
        const double vp = (i + 1 < n) ? V[o + ld] : 0.0;
        assemble_row<KIND>(i, n, vm, V[o], vp, rcoef, rw.e, rw.c, rw.d, rw.a, rw.b, rw.y);
      } else {
        rw.c = (double)C[o];
        rw.d = (double)D[o];
        rw.a = (double)A[o];
        rw.y = (double)Y[o];
        rw.e = rw.b = 0.0;
        if constexpr (KIND == 5 && SPARSE) {
          if (ol.kmax > kListScan && ol.kmax <= kListLds) {  // the staged list, rows ascending
            while (kc < s_lcnt[g] && s_lrow[kc * G + g] < i) ++kc;
            if (kc < s_lcnt[g] && s_lrow[kc * G + g] == i) {
              rw.e = (i >= 2) ? s_le[kc * G + g] : 0.0;
              rw.b = (i <= n - 3) ? s_lb[kc * G + g] : 0.0;
            }
          } else {
            for (int k = 0; k < ol.kmax; ++k) {
              const int64_t lo = (int64_t)k * ld + s;
              if (ol.row[lo] == i) {
                rw.e = (i >= 2) ? ol.e[lo] : 0.0;
                rw.b = (i <= n - 3) ? ol.b[lo] : 0.0;
              }
            }
          }
        } else if constexpr (KIND == 5) {
          rw.e = (double)E[o];
          rw.b = (double)B[o];
        }
      }
      return rw;
    };
    const int64_t plane = n * rpitch;
    const seq::Planes P{rws, rws + plane, rpitch, rws + (KIND == 5 ? 2 : 1) * plane, rpitch, s};
    const int64_t sb = seq::solve<KIND>(
        n, fetch, P,
        [&](int64_t i, double xv) {
          if constexpr (ACC)
            X[i * ld + s] = X[i * ld + s] + xv;
          else
            X[i * ld + s] = (TIO)xv;
        },
        [&](int64_t i) { return ((tiles_mask >> (uint32_t)(i / RT)) & 1u) != 0u; });
    st_coherent_i32(&info[s], sb < 0 ? 0 : (int32_t)(sb + 1));
  };
  if (T == 1) {
    if (tid < G && live && redo) redo_system(~0u);
    return;
  }
  // Departure, off the critical path: every tile read all maps before the
  // barrier after the exchange.  Wave 0 alone (it holds the info stores and
  // every lane with j == 0), so the other waves retire as soon as their x
  // stores are issued.  A tile that gave up adds its bit to the give-up
  // mask; a tile that read every map adds the systems it found bad to the
  // redo mask; then it departs.  Each departure waits for the returned value
  // of the mask update, so the last tile to leave sees every mask bit.
  if (tid < 64) {
    __builtin_amdgcn_s_waitcnt(kWaitVmem);  // this wave's info stores are in place
    const uint64_t bad_lanes = __ballot(tid < G && redo);
    unsigned last = 0;
    if (tid == 0) {
      const unsigned sysmask = (unsigned)(bad_lanes & ((1ull << G) - 1ull));
      unsigned before = 0;
      if (s_timeout)
        before = atomicOr(&cnt[4 * grp + 2], 1u << (unsigned)tile);
      else if (sysmask != 0u)
        before = atomicOr(&cnt[4 * grp + 3], sysmask);
      last = (before != ~0u && atomicAdd(&cnt[4 * grp + 1], 1u) == (unsigned)T - 1) ? 1u : 0u;
    }
    if (__builtin_amdgcn_readfirstlane(last)) {
      unsigned gave = 0, sysmask = 0;
      if (tid < G) {
        gave = ld_counter(&cnt[4 * grp + 2]);
        sysmask = ld_counter(&cnt[4 * grp + 3]);
      }
      if (tid < G && live && !list_bad) {
        if ((sysmask >> tid) & 1u)
          redo_system(~0u);
        else if (gave != 0u) {
          if (redo_gaveup)
            redo_system(gave);
          else
            st_coherent_i32(&info[s], kTimeout);
        }
      }
      if (tid == 0 && (gave | sysmask) != ~0u) {  // after the masks were read
        __hip_atomic_store(&cnt[4 * grp], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&cnt[4 * grp + 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&cnt[4 * grp + 2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&cnt[4 * grp + 3], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Long systems (more tiles than one group of blocks can exchange at once):
// three launches.
//   long_tile_kernel<FINISH=false>: every tile's local eliminations and tree,
//     tile map (and first bad row) to `maps`;
//   long_reduce_kernel: per system, the tile maps are folded left to right
//     within each lane's run of tiles, then merged up a tree across the lanes
//     of one wave; walking back down gives every tile its outer pairs
//     (`bounds`) and the system its info;
//   long_tile_kernel<FINISH=true>: every tile reloads its rows, repeats the
//     same local eliminations and tree (bitwise the same maps), walks down
//     from its outer pairs and writes x.
// Inputs are read twice; no per-row state goes through memory.
// ---------------------------------------------------------------------------
template <bool FINISH, typename TIO, int KIND, int M, int PW, int G>
__global__ __launch_bounds__(G * PW) void long_tile_kernel(
    int64_t n, int64_t batch, int64_t ld, const TIO* __restrict__ E,
    const TIO* __restrict__ C, const TIO* __restrict__ D,
    const TIO* __restrict__ A, const TIO* __restrict__ B,
    const TIO* __restrict__ Y, TIO* __restrict__ X, double* __restrict__ maps,
    const double* __restrict__ bounds, int64_t T, const int32_t* __restrict__ skip,
    const int32_t* __restrict__ info) {
  if (skip != nullptr && *skip) return;
  constexpr int NB = KIND == 5 ? 2 : 1;
  constexpr int RS = kRecSz<NB>;
  constexpr int XS = RS + 1;
  constexpr int RT = M * PW;
  __shared__ double s_node[(PW - 1) * G * RS];
  __shared__ int s_bad[G];
  const int tid = threadIdx.x;
  const int g = tid % G;
  const int j = tid / G;
  const int64_t grp = blockIdx.x / T, tile = blockIdx.x % T;
  const int64_t s = grp * G + g;
  const bool live = s < batch;
  const int64_t row_base = tile * RT;  // pointers rebased to the tile: 32-bit offsets inside it
  const int64_t shift = row_base * ld;
  const int64_t r0 = (int64_t)j * M;
  if (tid < G) s_bad[tid] = kBadNone;
  double c[M], d[M], a[M], y[M], e[M], b[M];
  load_chunk<KIND, M>(n, ld, s, live, r0, row_base, KIND == 5 ? E + shift : E, C + shift,
                      D + shift, A + shift, KIND == 5 ? B + shift : B, Y + shift, e, c, d, a,
                      b, y);
  double p[M], v[NB][M], w[NB][M];
  int bad;
  eliminate_chunk<KIND, M>(e, c, d, a, b, y, p, v, w, bad);
  Map<NB> mp = chunk_map<NB, M>(p, v, w);
  __syncthreads();
  if (!FINISH && bad < M && row_base + r0 + bad < n)
    atomicMin(&s_bad[g], (int)(row_base + r0 + bad + 1));
  tree_up<NB, PW, G, true>(mp, j, g, s_node, s_bad, M, row_base, n);
  const int64_t rec = (grp * T + tile) * G + g;
  if constexpr (!FINISH) {
    if (j == 0) {
      double* dst = maps + rec * XS;
      store_rec(mp, dst);
      dst[RS] = (double)s_bad[g];
    }
  } else {
    double xl[NB] = {}, xr[NB] = {};
    if (j == 0) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        xl[q] = bounds[rec * 2 * NB + q];
        xr[q] = bounds[rec * 2 * NB + NB + q];
      }
    }
    __syncthreads();
    tree_down<NB, PW, G, true>(xl, xr, j, g, s_node);
    // systems the reduction found bad are left to the sequential redo
    if (!(live && info[s] == seq::kRedo))
      write_chunk<NB, M>(n, ld, s, live, r0, row_base, p, v, w, xl, xr, X + shift);
  }
}

// The sequential redo of the systems marked seq::kRedo: lane t owns redo
// slot t (columns of the planes, pitch R) and takes systems t, t + R, ...
template <typename TIO, int KIND>
__global__ __launch_bounds__(64) void long_redo_kernel(
    int64_t n, int64_t batch, int64_t ld, const TIO* __restrict__ E, const TIO* __restrict__ C,
    const TIO* __restrict__ D, const TIO* __restrict__ A, const TIO* __restrict__ B,
    const TIO* __restrict__ Y, TIO* __restrict__ X, int32_t* __restrict__ info,
    double* __restrict__ planes, int64_t R, const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  const int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (t >= R) return;
  const int64_t plane = n * R;
  for (int64_t s = t; s < batch; s += R) {
    if (info[s] != seq::kRedo) continue;
    auto fetch = [&](int64_t i) {
      const int64_t o = i * ld + s;
      seq::Row rw;
      rw.e = (KIND == 5) ? (double)E[o] : 0.0;
      rw.c = (double)C[o];
      rw.d = (double)D[o];
      rw.a = (double)A[o];
      rw.b = (KIND == 5) ? (double)B[o] : 0.0;
      rw.y = (double)Y[o];
      return rw;
    };
    const seq::Planes P{planes, planes + plane, R, planes + (KIND == 5 ? 2 : 1) * plane, R, t};
    const int64_t sb = seq::solve<KIND>(
        n, fetch, P, [&](int64_t i, double xv) { X[i * ld + s] = (TIO)xv; },
        [](int64_t) { return true; });
    info[s] = sb < 0 ? 0 : (int32_t)(sb + 1);
  }
}

// One wave per system: lane l folds tiles [l*R, (l+1)*R) left to right
// (node records to `nodes`), then the 64 lane maps merge up a tree in LDS.
template <int KIND, int G>
__global__ __launch_bounds__(256) void long_reduce_kernel(
    int64_t n, int64_t batch, int64_t T, int64_t rows_per_tile,
    const double* __restrict__ maps, double* __restrict__ nodes,
    double* __restrict__ bounds, int32_t* __restrict__ info, const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  constexpr int NB = KIND == 5 ? 2 : 1;
  constexpr int RS = kRecSz<NB>;
  constexpr int XS = RS + 1;
  constexpr int WPB = 4;  // systems (waves) per block
  __shared__ double s_node[WPB * 63 * RS];
  __shared__ int s_bad[WPB];
  const int lane = threadIdx.x % 64;
  const int wv = threadIdx.x / 64;
  const int64_t s = (int64_t)blockIdx.x * WPB + wv;
  const bool live = s < batch;
  const int64_t grp = s / G, g = s % G;
  const int64_t R = (T + 63) / 64;
  const int64_t t0 = lane * R, t1 = (t0 + R < T) ? t0 + R : T;
  if (lane == 0) s_bad[wv] = kBadNone;
  __syncthreads();
  Map<NB> acc;
  zero_map(acc);
  int bad = kBadNone;
  if (live) {
    for (int64_t t = t0; t < t1; ++t) {
      const double* src = maps + ((grp * T + t) * G + g) * XS;
      Map<NB> m;
      load_rec(m, src);
      const double tb = src[RS];
      if (tb < (double)bad) bad = (int)tb;
      if (t == t0) {
        acc = m;
      } else {
        Node<NB> nd;
        if (!merge<NB>(acc, m, acc, nd)) {
          const int64_t row = t * rows_per_tile - NB;
          if (row < n && row + 1 < bad) bad = (int)(row + 1);
        }
        store_rec(nd, nodes + (s * T + t) * RS);
      }
    }
  }
  if (bad != kBadNone) atomicMin(&s_bad[wv], bad);
  // tree over the 64 runs of this wave (empty runs are zero maps)
  tree_up<NB, 64, 1>(acc, lane, 0, s_node + wv * 63 * RS, s_bad + wv, R * rows_per_tile, 0, n);
  double xl[NB], xr[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) xl[q] = xr[q] = 0.0;
  __syncthreads();
  tree_down<NB, 64, 1>(xl, xr, lane, 0, s_node + wv * 63 * RS);
  // walk back through this lane's run
  if (live && t0 < t1) {
    for (int64_t t = t1 - 1; t > t0; --t) {
      Node<NB> nd;
      load_rec(nd, nodes + (s * T + t) * RS);
      double ba[NB], tb[NB], u1[NB], u2[NB];
      mv<NB>(nd.G1, xl, u1);
      mv<NB>(nd.G2, xr, u2);
#pragma unroll
      for (int q = 0; q < NB; ++q) ba[q] = nd.g0[q] + u1[q] + u2[q];
      mv<NB>(nd.H1, xl, u1);
      mv<NB>(nd.H2, xr, u2);
#pragma unroll
      for (int q = 0; q < NB; ++q) tb[q] = nd.h0[q] + u1[q] + u2[q];
      double* dst = bounds + ((grp * T + t) * G + g) * 2 * NB;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        dst[q] = ba[q];
        dst[NB + q] = xr[q];
        xr[q] = tb[q];
      }
    }
    double* dst = bounds + ((grp * T + t0) * G + g) * 2 * NB;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      dst[q] = xl[q];
      dst[NB + q] = xr[q];
    }
  }
  __syncthreads();
  if (lane == 0 && live) info[s] = (s_bad[wv] == kBadNone) ? 0 : seq::kRedo;
}

struct Variant {
  int kind, M, PW, G, TMAX, WPE;  // WPE: waves per SIMD the register budget targets
};

// Compiled single-launch variants; index 0 of each kind is the default.
constexpr Variant kVariants[] = {
    {5, 32, 16, 16, 4, 1}, {5, 32, 16, 16, 8, 1}, {5, 16, 16, 16, 8, 1}, {5, 8, 32, 16, 8, 1},
    {3, 32, 16, 16, 4, 1}, {3, 32, 16, 16, 8, 1}, {3, 16, 16, 16, 8, 2}, {3, 16, 32, 16, 4, 2},
};
// FP32 storage with the compact (FP32) chunk state: twice the rows per lane
// (64), so the sweep batch is one round of blocks, and 32 systems per block,
// so a row of the tile is one 128-byte line of FP32 values.
constexpr Variant kCompact[] = {
    {5, 64, 8, 32, 4, 1}, {5, 64, 8, 32, 8, 1}, {3, 64, 8, 32, 4, 1}, {3, 64, 8, 32, 8, 1},
};
// Shape of the long-system path (both kinds).
constexpr int kLongM = 32, kLongPW = 16, kLongG = 16;

// Longest wait of a tile for the other tiles of its system, microseconds.
std::atomic<int64_t> g_exchange_wait_us{1000000};

// Workspace of a single-launch variant, in doubles: the meeting counters
// (4 per group) and the tile-map exchange when T > 1, then the planes of the
// sequential redo (alpha, beta, z for PD; alpha, z for TD), 256-byte aligned.
struct PartWs {
  int64_t xch, planes, total;
};
PartWs part_ws(int kind, int64_t n, int64_t batch, int64_t M, int64_t PW, int64_t G) {
  const int64_t RT = M * PW;
  const int64_t T = (n + RT - 1) / RT;
  const int64_t groups = (batch + G - 1) / G;
  const int64_t xs = (kind == 5 ? 20 : 6) + 1;
  PartWs W;
  // 4 unsigned counters per group, in a region sized for groups of 16 (the
  // smallest G) whatever this variant's G: every variant's counters then lie
  // in the same leading bytes, which every completed call leaves zero, so a
  // workspace may serve calls of different variants or dtypes in turn.
  W.xch = 2 * std::max(groups, (batch + 15) / 16);
  const int64_t head = (T > 1) ? W.xch + groups * T * G * xs : 0;
  W.planes = (head + 31) / 32 * 32;
  W.total = W.planes + (kind == 5 ? 3 : 2) * n * ws_ld(batch);
  return W;
}

template <typename TIO, int KIND, int M, int PW, int G, int TMAX, int WPE, bool SPARSE = false,
          bool ASM = false, typename TS = double, bool ACC = false>
hipError_t launch_cfg(int64_t n, int64_t batch, int64_t ld, const void* const* dg,
                      const void* y, void* x, int32_t* info, double* ws, hipStream_t st,
                      const int32_t* skip, Outer ol = Outer{0, nullptr, nullptr, nullptr},
                      double rcoef = 0.0, const int32_t* act = nullptr) {
  constexpr int RT = M * PW;
  const int T = (int)((n + RT - 1) / RT);
  const int64_t groups = (batch + G - 1) / G;
  const PartWs W = part_ws(KIND, n, batch, M, PW, G);
  unsigned* cnt = (T > 1) ? reinterpret_cast<unsigned*>(ws) : nullptr;
  double* xch = (T > 1) ? ws + W.xch : nullptr;
  hipLaunchKernelGGL((part_kernel<TIO, KIND, M, PW, G, TMAX, WPE, SPARSE, ASM, TS, ACC>),
                     dim3((unsigned)(groups * T)), dim3(G * PW), 0, st, n, batch, ld,
                     (const TIO*)dg[0], (const TIO*)dg[1], (const TIO*)dg[2], (const TIO*)dg[3],
                     (const TIO*)dg[4], (const TIO*)y, (TIO*)x, info, xch, cnt, T, skip, ol,
                     rcoef, (uint64_t)g_exchange_wait_us.load() * 100u, ws + W.planes,
                     ws_ld(batch), (int)(x != y), act);
  return hipGetLastError();
}

// Long-path workspace, in doubles: tile maps, outer pairs, fold nodes, then
// the planes of R redo slots (256-byte aligned).
struct LongWs {
  int64_t maps, bounds, nodes, planes, R, total;
};
LongWs long_ws(int kind, int64_t n, int64_t batch) {
  const int64_t NB = kind == 5 ? 2 : 1;
  const int64_t RS = 2 * NB + 4 * NB * NB;
  const int64_t RT = (int64_t)kLongM * kLongPW;
  const int64_t T = (n + RT - 1) / RT;
  const int64_t recs = (batch + kLongG - 1) / kLongG * T * kLongG;
  const int64_t np = kind == 5 ? 3 : 2;
  LongWs W;
  W.maps = 0;
  W.bounds = W.maps + recs * (RS + 1);
  W.nodes = W.bounds + recs * 2 * NB;
  W.planes = (W.nodes + batch * T * RS + 31) / 32 * 32;
  W.R = seq::redo_slots(np, n, batch);
  W.total = W.planes + np * n * W.R;
  return W;
}

template <typename TIO, int KIND>
hipError_t launch_long(int64_t n, int64_t batch, int64_t ld, const void* const* dg,
                       const void* y, void* x, int32_t* info, double* ws, hipStream_t st,
                       const int32_t* skip) {
  constexpr int M = kLongM, PW = kLongPW, G = kLongG;
  const int64_t RT = (int64_t)M * PW;
  const int64_t T = (n + RT - 1) / RT;
  const int64_t groups = (batch + G - 1) / G;
  const LongWs W = long_ws(KIND, n, batch);
  double* maps = ws + W.maps;
  double* bounds = ws + W.bounds;
  double* nodes = ws + W.nodes;
  const TIO* P[6] = {(const TIO*)dg[0], (const TIO*)dg[1], (const TIO*)dg[2],
                     (const TIO*)dg[3], (const TIO*)dg[4], (const TIO*)y};
  hipLaunchKernelGGL((long_tile_kernel<false, TIO, KIND, M, PW, G>), dim3((unsigned)(groups * T)),
                     dim3(G * PW), 0, st, n, batch, ld, P[0], P[1], P[2], P[3], P[4], P[5],
                     (TIO*)x, maps, bounds, T, skip, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((long_reduce_kernel<KIND, G>), dim3((unsigned)((batch + 3) / 4)), dim3(256),
                     0, st, n, batch, T, RT, maps, nodes, bounds, info, skip);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((long_tile_kernel<true, TIO, KIND, M, PW, G>), dim3((unsigned)(groups * T)),
                     dim3(G * PW), 0, st, n, batch, ld, P[0], P[1], P[2], P[3], P[4], P[5],
                     (TIO*)x, maps, bounds, T, skip, info);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((long_redo_kernel<TIO, KIND>), dim3((unsigned)((W.R + 63) / 64)), dim3(64),
                     0, st, n, batch, ld, P[0], P[1], P[2], P[3], P[4], P[5], (TIO*)x, info,
                     ws + W.planes, W.R, skip);
  return hipGetLastError();
}

const Variant* find_variant(int kind, int idx) {
  int k = 0;
  for (const Variant& v : kVariants)
    if (v.kind == kind && k++ == idx) return &v;
  return nullptr;
}

}  // namespace

void set_exchange_wait_us(int64_t us) { g_exchange_wait_us = us; }
int64_t exchange_wait_us() { return g_exchange_wait_us.load(); }

int part_variant_count(int kind) {
  int k = 0;
  for (const Variant& v : kVariants) k += v.kind == kind;
  return k;
}

bool part_variant_shape(int kind, int idx, int out[4]) {
  const Variant* v = find_variant(kind, idx);
  if (!v) return false;
  out[0] = v->M;
  out[1] = v->PW;
  out[2] = v->G;
  out[3] = v->TMAX;
  return true;
}

// FP32 storage is compiled for the first two variants of each kind.
static bool has_f32(int kind, int idx) {
  (void)kind;
  return idx == 0 || idx == 1;
}

static bool covers(const Variant* v, int64_t n, int64_t ld, int dtype) {
  const int64_t esz = dtype == 1 ? 4 : 8;
  if (n < 8 || n > (int64_t)v->M * v->PW * v->TMAX) return false;
  return (n + 1) * ld * esz < (int64_t(1) << 32);  // per-lane byte offsets are 32-bit
}

int part_pick(int kind, int idx, int64_t n, int64_t ld, int dtype) {
  const Variant* v = find_variant(kind, idx);
  if (v && covers(v, n, ld, dtype) && (dtype == 0 || has_f32(kind, idx))) return idx;
  for (int k = 0; k < part_variant_count(kind); ++k) {
    v = find_variant(kind, k);
    if (covers(v, n, ld, dtype) && (dtype == 0 || has_f32(kind, k))) return k;
  }
  return -1;
}

size_t part_counter_bytes(int kind, int idx, int64_t n, int64_t batch) {
  const Variant* v = find_variant(kind, idx);
  if (!v) return 0;
  const int64_t RT = (int64_t)v->M * v->PW;
  return (n + RT - 1) / RT > 1 ? (size_t)part_ws(kind, n, batch, v->M, v->PW, v->G).xch * 8 : 0;
}

size_t part_workspace_bytes(int kind, int idx, int64_t n, int64_t batch) {
  const Variant* v = find_variant(kind, idx);
  if (!v) return 0;
  return (size_t)part_ws(kind, n, batch, v->M, v->PW, v->G).total * 8;
}

hipError_t launch_part(int kind, int idx, int dtype, int64_t n, int64_t batch, int64_t ld,
                       const void* const dg[5], const void* y, void* x, int32_t* info,
                       double* ws, hipStream_t st, const int32_t* skip) {
  const Variant* v = find_variant(kind, idx);
  if (!v) return hipErrorInvalidValue;
#define BS_PV(TIO, K, MM, PP, GG, TT, WW)                                                \
  if (v->kind == K && v->M == MM && v->PW == PP && v->G == GG && v->TMAX == TT &&        \
      v->WPE == WW)                                                                      \
    return launch_cfg<TIO, K, MM, PP, GG, TT, WW>(n, batch, ld, dg, y, x, info, ws, st, skip);
  if (dtype == 0) {
    BS_PV(double, 5, 32, 16, 16, 4, 1) BS_PV(double, 5, 32, 16, 16, 8, 1)
    BS_PV(double, 5, 16, 16, 16, 8, 1) BS_PV(double, 5, 8, 32, 16, 8, 1)
    BS_PV(double, 3, 32, 16, 16, 4, 1) BS_PV(double, 3, 32, 16, 16, 8, 1)
    BS_PV(double, 3, 16, 16, 16, 8, 2) BS_PV(double, 3, 16, 32, 16, 4, 2)
  } else {
    BS_PV(float, 5, 32, 16, 16, 4, 1) BS_PV(float, 5, 32, 16, 16, 8, 1)
    BS_PV(float, 3, 32, 16, 16, 4, 1) BS_PV(float, 3, 32, 16, 16, 8, 1)
  }
#undef BS_PV
  return hipErrorInvalidValue;
}

const Variant* find_compact(int kind, int idx) {
  int k = 0;
  for (const Variant& v : kCompact)
    if (v.kind == kind && k++ == idx) return &v;
  return nullptr;
}

int compact_count(int kind) {
  int k = 0;
  for (const Variant& v : kCompact) k += v.kind == kind;
  return k;
}

int compact_pick(int kind, int idx, int64_t n, int64_t ld, int dtype) {
  const Variant* v = find_compact(kind, idx);
  if (v && covers(v, n, ld, dtype)) return idx;
  for (int k = 0; k < compact_count(kind); ++k)
    if (covers(find_compact(kind, k), n, ld, dtype)) return k;
  return -1;
}

size_t compact_counter_bytes(int kind, int idx, int64_t n, int64_t batch) {
  const Variant* v = find_compact(kind, idx);
  if (!v) return 0;
  const int64_t RT = (int64_t)v->M * v->PW;
  return (n + RT - 1) / RT > 1 ? (size_t)part_ws(kind, n, batch, v->M, v->PW, v->G).xch * 8 : 0;
}

size_t compact_workspace_bytes(int kind, int idx, int64_t n, int64_t batch) {
  const Variant* v = find_compact(kind, idx);
  if (!v) return 0;
  return (size_t)part_ws(kind, n, batch, v->M, v->PW, v->G).total * 8;
}

hipError_t launch_compact(int kind, int idx, int64_t n, int64_t batch, int64_t ld,
                          const void* const dg[5], const void* y, void* x, int32_t* info,
                          double* ws, hipStream_t st, const int32_t* skip) {
  const Variant* v = find_compact(kind, idx);
  if (!v) return hipErrorInvalidValue;
#define BS_PC(K, MM, PP, GG, TT, WW)                                                     \
  if (v->kind == K && v->M == MM && v->PW == PP && v->G == GG && v->TMAX == TT &&        \
      v->WPE == WW)                                                                      \
    return launch_cfg<float, K, MM, PP, GG, TT, WW, false, false, float>(                \
        n, batch, ld, dg, y, x, info, ws, st, skip);
  BS_PC(5, 64, 8, 32, 4, 1) BS_PC(5, 64, 8, 32, 8, 1)
  BS_PC(3, 64, 8, 32, 4, 1) BS_PC(3, 64, 8, 32, 8, 1)
#undef BS_PC
  return hipErrorInvalidValue;
}

hipError_t launch_compact_f64(int kind, int idx, int64_t n, int64_t batch, int64_t ld,
                              const double* const dg[5], const double* y, double* x,
                              int32_t* info, double* ws, hipStream_t st, const int32_t* skip,
                              bool acc, const int32_t* act) {
  const Variant* v = find_compact(kind, idx);
  if (!v) return hipErrorInvalidValue;
  const void* const* d = reinterpret_cast<const void* const*>(dg);
#define BS_PF(K, MM, PP, GG, TT, WW)                                                        \
  if (v->kind == K && v->M == MM && v->PW == PP && v->G == GG && v->TMAX == TT &&           \
      v->WPE == WW)                                                                         \
    return acc ? launch_cfg<double, K, MM, PP, GG, TT, WW, false, false, float, true>(      \
                     n, batch, ld, d, y, x, info, ws, st, skip, Outer{0, nullptr, nullptr,  \
                     nullptr}, 0.0, act)                                                    \
               : launch_cfg<double, K, MM, PP, GG, TT, WW, false, false, float, false>(     \
                     n, batch, ld, d, y, x, info, ws, st, skip, Outer{0, nullptr, nullptr,  \
                     nullptr}, 0.0, act);
  BS_PF(5, 64, 8, 32, 4, 1) BS_PF(5, 64, 8, 32, 8, 1)
  BS_PF(3, 64, 8, 32, 4, 1) BS_PF(3, 64, 8, 32, 8, 1)
#undef BS_PF
  return hipErrorInvalidValue;
}

// MNPDM with the rows split over lanes: the first two PD variants.
int part_mnpdm_pick(int idx, int64_t n, int64_t ld) {
  const int k = part_pick(5, idx, n, ld, 0);
  if (k == 0 || k == 1) return k;
  for (int q = 0; q < 2; ++q)
    if (covers(find_variant(5, q), n, ld, 0)) return q;
  return -1;
}

hipError_t launch_part_mnpdm(int idx, int64_t n, int64_t batch, int64_t ld,
                             const double* const cda[3], int32_t kmax, const int32_t* orow,
                             const double* oe, const double* ob, const double* y, double* x,
                             int32_t* info, double* ws, hipStream_t st) {
  const void* dg[5] = {nullptr, cda[0], cda[1], cda[2], nullptr};
  const Outer ol{kmax, orow, oe, ob};
  if (idx == 0)
    return launch_cfg<double, 5, 32, 16, 16, 4, 1, true>(n, batch, ld, dg, y, x, info, ws, st,
                                                         nullptr, ol);
  if (idx == 1)
    return launch_cfg<double, 5, 32, 16, 16, 8, 1, true>(n, batch, ld, dg, y, x, info, ws, st,
                                                         nullptr, ol);
  return hipErrorInvalidValue;
}

// Assembled ADI sweep on the split kernels: the first two variants of `kind`.
int part_adi_pick(int kind, int idx, int64_t n, int64_t ld) {
  const int k = part_pick(kind, idx, n, ld, 0);
  if (k == 0 || k == 1) return k;
  for (int q = 0; q < 2; ++q)
    if (covers(find_variant(kind, q), n, ld, 0)) return q;
  return -1;
}

hipError_t launch_part_adi(int kind, int idx, int64_t n, int64_t batch, int64_t ld, double r,
                           const double* v, double* x, int32_t* info, double* ws,
                           hipStream_t st) {
  const void* dg[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const Outer none{0, nullptr, nullptr, nullptr};
#define BS_PA(K, TT)                                                                        \
  return launch_cfg<double, K, 32, 16, 16, TT, 1, false, true>(n, batch, ld, dg, v, x, info, \
                                                               ws, st, nullptr, none, r);
  if (kind == 5 && idx == 0) { BS_PA(5, 4) }
  if (kind == 5 && idx == 1) { BS_PA(5, 8) }
  if (kind == 3 && idx == 0) { BS_PA(3, 4) }
  if (kind == 3 && idx == 1) { BS_PA(3, 8) }
#undef BS_PA
  return hipErrorInvalidValue;
}

bool long_supported(int64_t n, int64_t ld, int dtype) {
  const int64_t esz = dtype == 1 ? 4 : 8;
  return n >= 8 && (int64_t)(kLongM * kLongPW + 1) * ld * esz < (int64_t(1) << 32);
}

size_t long_workspace_bytes(int kind, int64_t n, int64_t batch) {
  return (size_t)long_ws(kind, n, batch).total * 8;
}

hipError_t launch_long_path(int kind, int dtype, int64_t n, int64_t batch, int64_t ld,
                            const void* const dg[5], const void* y, void* x, int32_t* info,
                            double* ws, hipStream_t st, const int32_t* skip) {
  if (dtype == 0)
    return kind == 5 ? launch_long<double, 5>(n, batch, ld, dg, y, x, info, ws, st, skip)
                     : launch_long<double, 3>(n, batch, ld, dg, y, x, info, ws, st, skip);
  return kind == 5 ? launch_long<float, 5>(n, batch, ld, dg, y, x, info, ws, st, skip)
                   : launch_long<float, 3>(n, batch, ld, dg, y, x, info, ws, st, skip);
}

}  // namespace bs
