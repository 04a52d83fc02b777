// varlen.hip -- uneven batches: NPDM / NTDM for systems of different lengths
// in one solve (the N lines of an ADI sweep on an irregular domain, or the
// sweeps of many grids at once; Sec. 1 of Veneva & Ayriyan, arXiv:1804.09666
// solves each such system independently).
//
// Layout.  Systems are sorted by length (longest first) and packed in groups
// of 16; group g stores its systems batch-interleaved as an [n_g][16] block
// (n_g = its longest member), so one row of a group is one 128-byte line and
// sorting keeps the padding of a group small.  Row r of system i lives at
// offset[i] + 16 r of every array (offset from bs_varlen_layout).
//
// Solve.  The rows of every group are cut into tiles of RT = M x PW rows and
// solved by the partitioned elimination of direct_part.hip in three launches
// over ALL groups at once (the grid enumerates every (group, tile) pair):
//   tile pass   -- every tile's chunk eliminations and in-block tree, tile
//                  map to the workspace;
//   reduce      -- one wave per system folds its tile maps and hands every
//                  tile its outer pairs;
//   finish pass -- every tile repeats its local work (bitwise) and writes x.
// Rows past a system's own length are identity rows: never read, never
// written.  The tile shape is a compiled variant; bs_varlen_tune times each
// on the caller's data and returns the fastest.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "bandsolve.h"
#include "seq_core.h"
#include "split_core.h"

namespace bs {
namespace {

using namespace split;

constexpr int kVG = 16;  // systems per group
constexpr int kNV = 3;   // compiled tile shapes

struct Shape {
  int M, PW;
};
constexpr Shape kShapes[kNV] = {{32, 16}, {16, 16}, {32, 8}};

// Device tables (one buffer, see table_layout).
struct VarTab {
  const int64_t* goff;  // [G] element offset of group g's block
  const int64_t* tpre;  // [G + 1] first tile of each group, this shape
  const int32_t* gn;    // [G] rows of the group
  const int32_t* sn;    // [16 G] rows of the system in each slot (0 = empty)
  int64_t groups;
};

__device__ inline int64_t group_of(const int64_t* __restrict__ tpre, int64_t groups, int64_t b) {
  int64_t lo = 0, hi = groups;  // tpre[lo] <= b < tpre[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (tpre[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <bool FINISH, int KIND, int M, int PW>
__global__ __launch_bounds__(kVG * PW) void varlen_tile_kernel(
    VarTab tab, const double* __restrict__ E, const double* __restrict__ C,
    const double* __restrict__ D, const double* __restrict__ A, const double* __restrict__ B,
    const double* __restrict__ Y, double* __restrict__ X, double* __restrict__ maps,
    const double* __restrict__ bounds, const int32_t* __restrict__ info) {
  constexpr int G = kVG;
  constexpr int NB = KIND == 5 ? 2 : 1;
  constexpr int RS = kRecSz<NB>;
  constexpr int XS = RS + 1;
  constexpr int RT = M * PW;
  __shared__ double s_node[(PW - 1) * G * RS];
  __shared__ int s_bad[G];
  const int tid = threadIdx.x;
  const int g = tid % G;
  const int j = tid / G;
  const int64_t grp = group_of(tab.tpre, tab.groups, blockIdx.x);
  const int64_t tile = blockIdx.x - tab.tpre[grp];
  const int64_t ng = tab.gn[grp];
  const int64_t ns = tab.sn[grp * G + g];
  const bool live = ns > 0;
  const int64_t row_base = tile * RT;
  const int64_t shift = tab.goff[grp] + row_base * G;  // element offset of the tile's row 0
  const int64_t r0 = (int64_t)j * M;
  if (tid < G) s_bad[tid] = kBadNone;
  double c[M], d[M], a[M], y[M], e[M], b[M];
  load_chunk<KIND, M>(ns, G, g, live, r0, row_base, KIND == 5 ? E + shift : E, C + shift,
                      D + shift, A + shift, KIND == 5 ? B + shift : B, Y + shift, e, c, d, a, b,
                      y);
  double p[M], v[NB][M], w[NB][M];
  int bad;
  eliminate_chunk<KIND, M>(e, c, d, a, b, y, p, v, w, bad);
  Map<NB> mp = chunk_map<NB, M>(p, v, w);
  __syncthreads();
  if (!FINISH && bad < M && row_base + r0 + bad < ns)
    atomicMin(&s_bad[g], (int)(row_base + r0 + bad + 1));
  tree_up<NB, PW, G, true>(mp, j, g, s_node, s_bad, M, row_base, ng);
  const int64_t rec = (tab.tpre[grp] + tile) * G + g;
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
    if (!(live && info[grp * G + g] == seq::kRedo))
      write_chunk<NB, M>(ns, G, g, live, r0, row_base, p, v, w, xl, xr, X + shift);
  }
}

// One wave per system slot: lane l folds tiles [l R, (l+1) R) left to right,
// then the 64 lane maps merge up a tree in LDS; walking back gives every tile
// its outer pairs.
template <int KIND>
__global__ __launch_bounds__(256) void varlen_reduce_kernel(VarTab tab, int64_t rows_per_tile,
                                                            const double* __restrict__ maps,
                                                            double* __restrict__ nodes,
                                                            double* __restrict__ bounds,
                                                            int32_t* __restrict__ info) {
  constexpr int G = kVG;
  constexpr int NB = KIND == 5 ? 2 : 1;
  constexpr int RS = kRecSz<NB>;
  constexpr int XS = RS + 1;
  constexpr int WPB = 4;
  __shared__ double s_node[WPB * 63 * RS];
  __shared__ int s_bad[WPB];
  const int lane = threadIdx.x % 64;
  const int wv = threadIdx.x / 64;
  const int64_t slot = (int64_t)blockIdx.x * WPB + wv;
  const bool inside = slot < tab.groups * G;
  const int64_t ns = inside ? tab.sn[slot] : 0;
  const bool live = ns > 0;
  const int64_t grp = inside ? slot / G : 0, g = slot % G;
  const int64_t T = inside ? tab.tpre[grp + 1] - tab.tpre[grp] : 0;
  const int64_t rec0 = inside ? tab.tpre[grp] * G + g : 0;  // record of tile t: rec0 + t G
  const int64_t R = (T + 63) / 64;
  const int64_t t0 = lane * R, t1 = (t0 + R < T) ? t0 + R : T;
  if (lane == 0) s_bad[wv] = kBadNone;
  __syncthreads();
  Map<NB> acc;
  zero_map(acc);
  int bad = kBadNone;
  if (live) {
    for (int64_t t = t0; t < t1; ++t) {
      const double* src = maps + (rec0 + t * G) * XS;
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
          if (row < ns && row + 1 < bad) bad = (int)(row + 1);
        }
        store_rec(nd, nodes + (rec0 + t * G) * RS);
      }
    }
  }
  if (bad != kBadNone) atomicMin(&s_bad[wv], bad);
  tree_up<NB, 64, 1>(acc, lane, 0, s_node + wv * 63 * RS, s_bad + wv, R * rows_per_tile, 0, ns);
  double xl[NB], xr[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) xl[q] = xr[q] = 0.0;
  __syncthreads();
  tree_down<NB, 64, 1>(xl, xr, lane, 0, s_node + wv * 63 * RS);
  if (live && t0 < t1) {
    for (int64_t t = t1 - 1; t > t0; --t) {
      Node<NB> nd;
      load_rec(nd, nodes + (rec0 + t * G) * RS);
      double ba[NB], tb[NB], u1[NB], u2[NB];
      mv<NB>(nd.G1, xl, u1);
      mv<NB>(nd.G2, xr, u2);
#pragma unroll
      for (int q = 0; q < NB; ++q) ba[q] = nd.g0[q] + u1[q] + u2[q];
      mv<NB>(nd.H1, xl, u1);
      mv<NB>(nd.H2, xr, u2);
#pragma unroll
      for (int q = 0; q < NB; ++q) tb[q] = nd.h0[q] + u1[q] + u2[q];
      double* dst = bounds + (rec0 + t * G) * 2 * NB;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        dst[q] = ba[q];
        dst[NB + q] = xr[q];
        xr[q] = tb[q];
      }
    }
    double* dst = bounds + (rec0 + t0 * G) * 2 * NB;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      dst[q] = xl[q];
      dst[NB + q] = xr[q];
    }
  }
  __syncthreads();
  if (lane == 0 && live) info[slot] = (s_bad[wv] == kBadNone) ? 0 : seq::kRedo;
}

// The sequential redo of the systems marked seq::kRedo: lane t owns redo
// slot t (plane columns, pitch R) and takes system slots t, t + R, ...
template <int KIND>
__global__ __launch_bounds__(64) void varlen_redo_kernel(
    VarTab tab, const double* __restrict__ E, const double* __restrict__ C,
    const double* __restrict__ D, const double* __restrict__ A, const double* __restrict__ B,
    const double* __restrict__ Y, double* __restrict__ X, int32_t* __restrict__ info,
    double* __restrict__ planes, int64_t R, int64_t nmax) {
  const int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (t >= R) return;
  const int64_t plane = nmax * R;
  for (int64_t slot = t; slot < tab.groups * kVG; slot += R) {
    const int64_t ns = tab.sn[slot];
    if (ns <= 0 || info[slot] != seq::kRedo) continue;
    const int64_t base = tab.goff[slot / kVG] + slot % kVG;  // row r at base + 16 r
    auto fetch = [&](int64_t i) {
      const int64_t o = base + i * kVG;
      seq::Row rw;
      rw.e = (KIND == 5) ? E[o] : 0.0;
      rw.c = C[o];
      rw.d = D[o];
      rw.a = A[o];
      rw.b = (KIND == 5) ? B[o] : 0.0;
      rw.y = Y[o];
      return rw;
    };
    const seq::Planes P{planes, planes + plane, R, planes + (KIND == 5 ? 2 : 1) * plane, R, t};
    const int64_t sb = seq::solve<KIND>(
        ns, fetch, P, [&](int64_t i, double xv) { X[base + i * kVG] = xv; },
        [](int64_t) { return true; });
    info[slot] = sb < 0 ? 0 : (int32_t)(sb + 1);
  }
}

// ---------------------------------------------------------------- host ---
struct TableLayout {
  size_t goff, tpre, gn, sn, total;  // byte offsets
};
TableLayout table_layout(int64_t groups) {
  TableLayout L;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  size_t o = 0;
  L.goff = o; o = up(o + (size_t)groups * 8);
  L.tpre = o; o = up(o + (size_t)(groups + 1) * 8 * kNV);
  L.gn = o;   o = up(o + (size_t)groups * 4);
  L.sn = o;   o = up(o + (size_t)groups * kVG * 4);
  L.total = o;
  return L;
}

VarTab dev_tab(const bs_varlen_info* vi, const void* table, int variant) {
  const TableLayout L = table_layout(vi->groups);
  const char* base = static_cast<const char*>(table);
  VarTab t;
  t.goff = reinterpret_cast<const int64_t*>(base + L.goff);
  t.tpre = reinterpret_cast<const int64_t*>(base + L.tpre) + (size_t)(vi->groups + 1) * variant;
  t.gn = reinterpret_cast<const int32_t*>(base + L.gn);
  t.sn = reinterpret_cast<const int32_t*>(base + L.sn);
  t.groups = vi->groups;
  return t;
}

struct WsLayout {
  size_t maps, bounds, nodes, planes, total;  // in doubles
  int64_t R;                                  // redo slots
};
WsLayout ws_layout(int kind, int64_t tiles, int64_t count, int64_t nmax) {
  const int64_t NB = kind == 5 ? 2 : 1, RS = 2 * NB + 4 * NB * NB;
  const int64_t np = kind == 5 ? 3 : 2;
  const int64_t recs = tiles * kVG;
  WsLayout W;
  W.maps = 0;
  W.bounds = W.maps + recs * (RS + 1);
  W.nodes = W.bounds + recs * 2 * NB;
  W.planes = (W.nodes + recs * RS + 31) / 32 * 32;
  W.R = seq::redo_slots(np, nmax, count);
  W.total = W.planes + (size_t)(np * nmax * W.R);
  return W;
}

template <int KIND, int M, int PW>
hipError_t launch_shape(const VarTab& tab, int64_t tiles, int64_t slots, const WsLayout& W,
                        int64_t nmax, const void* const dg[5], const double* y, double* x,
                        int32_t* info, double* ws, hipStream_t st) {
  const double* P[5] = {static_cast<const double*>(dg[0]), static_cast<const double*>(dg[1]),
                        static_cast<const double*>(dg[2]), static_cast<const double*>(dg[3]),
                        static_cast<const double*>(dg[4])};
  hipLaunchKernelGGL((varlen_tile_kernel<false, KIND, M, PW>), dim3((unsigned)tiles),
                     dim3(kVG * PW), 0, st, tab, P[0], P[1], P[2], P[3], P[4], y, x,
                     ws + W.maps, ws + W.bounds, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((varlen_reduce_kernel<KIND>), dim3((unsigned)((slots + 3) / 4)), dim3(256),
                     0, st, tab, (int64_t)M * PW, ws + W.maps, ws + W.nodes, ws + W.bounds,
                     info);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((varlen_tile_kernel<true, KIND, M, PW>), dim3((unsigned)tiles),
                     dim3(kVG * PW), 0, st, tab, P[0], P[1], P[2], P[3], P[4], y, x,
                     ws + W.maps, ws + W.bounds, info);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((varlen_redo_kernel<KIND>), dim3((unsigned)((W.R + 63) / 64)), dim3(64), 0,
                     st, tab, P[0], P[1], P[2], P[3], P[4], y, x, info, ws + W.planes, W.R, nmax);
  return hipGetLastError();
}

hipError_t launch_varlen(int kind, int variant, const bs_varlen_info* vi, const void* table,
                         const void* const dg[5], const double* y, double* x, int32_t* info,
                         double* ws, hipStream_t st) {
  const VarTab tab = dev_tab(vi, table, variant);
  const int64_t tiles = vi->tiles[variant], slots = vi->groups * kVG;
  const WsLayout W = ws_layout(kind, tiles, vi->count, vi->nmax);
#define BS_VL(K, V, MM, PP)                                                                   \
  if (kind == K && variant == V)                                                              \
    return launch_shape<K, MM, PP>(tab, tiles, slots, W, vi->nmax, dg, y, x, info, ws, st);
  BS_VL(5, 0, 32, 16) BS_VL(5, 1, 16, 16) BS_VL(5, 2, 32, 8)
  BS_VL(3, 0, 32, 16) BS_VL(3, 1, 16, 16) BS_VL(3, 2, 32, 8)
#undef BS_VL
  return hipErrorInvalidValue;
}

bool info_ok(const bs_varlen_info* vi) {
  if (vi == nullptr || vi->count < 1 || vi->groups < 1 || vi->groups > (int64_t(1) << 26) ||
      vi->nmax < 8 || vi->nmax >= (int64_t(1) << 31))
    return false;
  for (int v = 0; v < kNV; ++v)
    if (vi->tiles[v] < vi->groups || vi->tiles[v] > (int64_t(1) << 31)) return false;
  return true;
}

bool aligned8(const void* p) { return p != nullptr && (reinterpret_cast<uintptr_t>(p) & 7) == 0; }

}  // namespace
}  // namespace bs

extern "C" {

int32_t bs_varlen_variants(void) { return bs::kNV; }

int32_t bs_varlen_variant_shape(int32_t variant, int32_t shape[2]) {
  if (variant < 0 || variant >= bs::kNV || shape == nullptr) return BS_EINVAL;
  shape[0] = bs::kShapes[variant].M;
  shape[1] = bs::kShapes[variant].PW;
  return BS_OK;
}

int32_t bs_varlen_layout(int64_t count, const int64_t* n, int64_t* offset, int32_t* slot,
                         void* table, bs_varlen_info* info) {
  using namespace bs;
  if (count < 1 || n == nullptr || info == nullptr) return BS_EINVAL;
  for (int64_t i = 0; i < count; ++i)
    if (n[i] < 8 || n[i] >= (int64_t(1) << 31)) return BS_EINVAL;
  std::vector<int64_t> order((size_t)count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [n](int64_t a, int64_t b) { return n[a] > n[b]; });
  const int64_t groups = (count + kVG - 1) / kVG;
  std::vector<int64_t> goff((size_t)groups), tpre((size_t)(groups + 1) * kNV);
  std::vector<int32_t> gn((size_t)groups), sn((size_t)groups * kVG, 0);
  int64_t elems = 0;
  for (int64_t g = 0; g < groups; ++g) {
    gn[g] = (int32_t)n[order[g * kVG]];  // sorted: the first member is the longest
    goff[g] = elems;
    elems += (int64_t)gn[g] * kVG;
  }
  info->count = count;
  info->groups = groups;
  info->elems = elems;
  info->nmax = gn[0];
  for (int v = 0; v < kNV; ++v) {
    const int64_t RT = (int64_t)kShapes[v].M * kShapes[v].PW;
    int64_t t = 0;
    for (int64_t g = 0; g < groups; ++g) {
      tpre[(size_t)(groups + 1) * v + g] = t;
      t += (gn[g] + RT - 1) / RT;
    }
    tpre[(size_t)(groups + 1) * v + groups] = t;
    info->tiles[v] = t;
  }
  for (int v = kNV; v < 4; ++v) info->tiles[v] = 0;
  const TableLayout L = table_layout(groups);
  info->table_bytes = L.total;
  for (int64_t k = 0; k < count; ++k) {
    const int64_t i = order[k], g = k / kVG, lane = k % kVG;
    sn[k] = (int32_t)n[i];
    if (offset) offset[i] = goff[g] + lane;
    if (slot) slot[i] = (int32_t)k;
  }
  if (table != nullptr) {
    char* base = static_cast<char*>(table);
    memset(base, 0, L.total);
    memcpy(base + L.goff, goff.data(), goff.size() * 8);
    memcpy(base + L.tpre, tpre.data(), tpre.size() * 8);
    memcpy(base + L.gn, gn.data(), gn.size() * 4);
    memcpy(base + L.sn, sn.data(), sn.size() * 4);
  }
  return BS_OK;
}

size_t bs_varlen_workspace_bytes(int32_t kind, const bs_varlen_info* info, int32_t variant) {
  if ((kind != 3 && kind != 5) || !bs::info_ok(info) || variant < 0 || variant >= bs::kNV)
    return (size_t)-1;
  return bs::ws_layout(kind, info->tiles[variant], info->count, info->nmax).total * 8;
}

int32_t band_solve_varlen(int32_t kind, const bs_varlen_info* vinfo, const void* table,
                          int32_t variant, const void* const diags[5], const void* rhs, void* x,
                          int32_t* info, void* workspace, size_t ws_bytes, void* stream) {
  using namespace bs;
  if ((kind != 3 && kind != 5) || !info_ok(vinfo) || variant < 0 || variant >= kNV)
    return BS_EINVAL;
  if (table == nullptr || (reinterpret_cast<uintptr_t>(table) & 255) != 0 || diags == nullptr)
    return BS_EINVAL;
  for (int k = 0; k < 5; ++k)
    if ((kind == 5 || (k >= 1 && k <= 3)) && !aligned8(diags[k])) return BS_EINVAL;
  if (!aligned8(rhs) || !aligned8(x) || info == nullptr) return BS_EINVAL;
  const size_t need = bs_varlen_workspace_bytes(kind, vinfo, variant);
  if (ws_bytes < need) return BS_EWORKSPACE;
  if (!aligned8(workspace)) return BS_EINVAL;
  int devices = 0;
  if (hipGetDeviceCount(&devices) != hipSuccess || devices < 1) return BS_ENODEV;
  return launch_varlen(kind, variant, vinfo, table, diags, static_cast<const double*>(rhs),
                       static_cast<double*>(x), info, static_cast<double*>(workspace),
                       static_cast<hipStream_t>(stream)) == hipSuccess
             ? BS_OK
             : BS_ELAUNCH;
}

int32_t bs_varlen_tune(int32_t kind, const bs_varlen_info* vinfo, const void* table,
                       const void* const diags[5], const void* rhs, void* x, int32_t* info,
                       void* workspace, size_t ws_bytes, int32_t reps, float* ms,
                       int32_t* best, void* stream) {
  using namespace bs;
  if (reps < 1 || best == nullptr) return BS_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return BS_ELAUNCH;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return BS_ELAUNCH;
  }
  int32_t status = BS_OK;
  float best_ms = -1.0f;
  *best = -1;
  for (int v = 0; v < kNV && status == BS_OK; ++v) {
    status = band_solve_varlen(kind, vinfo, table, v, diags, rhs, x, info, workspace, ws_bytes,
                               stream);  // warm-up (and argument checks)
    if (status != BS_OK) break;
    if (hipEventRecord(a, st) != hipSuccess) status = BS_ELAUNCH;
    for (int r = 0; r < reps && status == BS_OK; ++r)
      status = band_solve_varlen(kind, vinfo, table, v, diags, rhs, x, info, workspace,
                                 ws_bytes, stream);
    if (status != BS_OK) break;
    float t = 0.0f;
    if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&t, a, b) != hipSuccess) {
      status = BS_ELAUNCH;
      break;
    }
    t /= (float)reps;
    if (ms) ms[v] = t;
    if (best_ms < 0.0f || t < best_ms) {
      best_ms = t;
      *best = v;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return status;
}

}  // extern "C"
