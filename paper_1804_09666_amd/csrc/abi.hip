// abi.hip -- the exported C ABI of libbandsolve (declared in
// include/bandsolve.h): host-side argument checks, workspace sizing and the
// choice of kernel, then an asynchronous launch on the caller's stream.
//
// Every check that can fail happens before the first HIP call, so a rejected
// call never touches the device (and can be exercised on a machine without a
// GPU).
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>

#include "bandsolve.h"
#include "bs_internal.h"

namespace {

constexpr int64_t kMaxElems = int64_t(1) << 50;  // guards n*ld overflow

bool aligned(const void* p, size_t a) {
  return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

bool shape_ok(int64_t n, int64_t batch, int64_t ld) {
  if (n < 1 || batch < 1 || ld < batch) return false;
  if (n >= (int64_t(1) << 31) - 1 || batch >= (int64_t(1) << 31)) return false;
  if (ld > kMaxElems / n) return false;
  return true;
}

bool kind_ok(int32_t kind) { return kind == 3 || kind == 5; }

size_t elem_size(int32_t dtype) { return dtype == BS_F32 ? 4 : 8; }

bool array_ok(const void* p, int32_t dtype) {
  return p != nullptr && aligned(p, elem_size(dtype));
}

// Diagonals a kind reads: PD all five, TD c, d, a.
bool diags_ok(int32_t kind, const void* const diags[5], int32_t dtype) {
  if (diags == nullptr) return false;
  for (int k = 0; k < 5; ++k) {
    const bool needed = (kind == 5) || (k >= 1 && k <= 3);
    if (needed && !array_ok(diags[k], dtype)) return false;
  }
  return true;
}

bs::Diags as_diags(int32_t kind, const void* const diags[5]) {
  bs::Diags A;
  A.e = kind == 5 ? static_cast<const double*>(diags[0]) : nullptr;
  A.c = static_cast<const double*>(diags[1]);
  A.d = static_cast<const double*>(diags[2]);
  A.a = static_cast<const double*>(diags[3]);
  A.b = kind == 5 ? static_cast<const double*>(diags[4]) : nullptr;
  return A;
}

// Tuning options (process-wide).
std::atomic<int64_t> g_direct_path{0};
std::atomic<int64_t> g_pd_variant{0}, g_td_variant{0};
std::atomic<int64_t> g_sip_path{0};
std::atomic<int64_t> g_f32_state{1};

int part_idx(int32_t kind) { return (int)(kind == 5 ? g_pd_variant.load() : g_td_variant.load()); }

}  // namespace

namespace bs {
namespace {

// Which fused kernel solves (kind, dtype, n, ld) under the current options.
enum class Route { kLane, kPart, kCompact, kLong, kNone };

Route route(int kind, int dtype, int64_t n, int64_t ld, int* idx) {
  *idx = -1;
  const int64_t fs = g_f32_state.load();
  if (g_direct_path.load() != 1 && dtype == BS_F32 && fs != 0) {
    *idx = compact_pick(kind, fs >= 2 ? (int)(fs - 2) : 0, n, ld);
    if (*idx >= 0) return Route::kCompact;
  }
  if (g_direct_path.load() != 1) {
    *idx = part_pick(kind, part_idx(kind), n, ld, dtype);
    if (*idx >= 0) return Route::kPart;
    if (long_supported(n, ld, dtype)) return Route::kLong;
  }
  return dtype == BS_F64 ? Route::kLane : Route::kNone;
}

}  // namespace

bool f32_compact_state() { return g_f32_state.load() != 0 && g_direct_path.load() != 1; }

bool direct_supported(int kind, int dtype, int64_t n, int64_t ld) {
  int idx;
  return route(kind, dtype, n, ld, &idx) != Route::kNone;
}

size_t direct_ws_bytes(int kind, int dtype, int64_t n, int64_t batch, int64_t ld) {
  int idx;
  switch (route(kind, dtype, n, ld, &idx)) {
    case Route::kPart: return part_workspace_bytes(kind, idx, n, batch);
    case Route::kCompact: return compact_workspace_bytes(kind, idx, n, batch);
    case Route::kLong: return long_workspace_bytes(kind, n, batch);
    case Route::kLane: return (size_t)((kind == 5 ? 2 : 1) * n * ws_ld(batch)) * 8;
    default: return 0;
  }
}

size_t direct_counter_bytes(int kind, int dtype, int64_t n, int64_t batch, int64_t ld) {
  int idx;
  switch (route(kind, dtype, n, ld, &idx)) {
    case Route::kPart: return part_counter_bytes(kind, idx, n, batch);
    case Route::kCompact: return compact_counter_bytes(kind, idx, n, batch);
    default: return 0;
  }
}

hipError_t launch_direct(int kind, int dtype, int64_t n, int64_t batch, int64_t ld,
                         const void* const dg[5], const void* y, void* x, int32_t* info,
                         void* ws, hipStream_t st, const int32_t* skip) {
  int idx;
  double* w = static_cast<double*>(ws);
  switch (route(kind, dtype, n, ld, &idx)) {
    case Route::kPart:
      return launch_part(kind, idx, dtype, n, batch, ld, dg, y, x, info, w, st, skip);
    case Route::kCompact:
      return launch_compact(kind, idx, n, batch, ld, dg, y, x, info, w, st, skip);
    case Route::kLong:
      return launch_long_path(kind, dtype, n, batch, ld, dg, y, x, info, w, st, skip);
    case Route::kLane: {
      if (skip != nullptr) return hipErrorInvalidValue;  // lane kernels take no skip flag
      Diags A = as_diags(kind, dg);
      if (kind == 5)
        return launch_npdm_lane(n, batch, ld, A, static_cast<const double*>(y),
                                static_cast<double*>(x), info, w, st);
      return launch_ntdm_lane(n, batch, ld, A, static_cast<const double*>(y),
                              static_cast<double*>(x), info, w, st);
    }
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace bs

namespace {

int32_t launched(hipError_t e) { return e == hipSuccess ? BS_OK : BS_ELAUNCH; }

// Split-row MNPDM variant for (n, ld) under the current options, or -1 for
// one lane per system.
int mnpdm_part_idx(int64_t n, int64_t ld) {
  if (g_direct_path.load() == 1) return -1;
  return bs::part_mnpdm_pick(part_idx(5), n, ld);
}

bool have_device() {
  int count = 0;
  return hipGetDeviceCount(&count) == hipSuccess && count > 0;
}

}  // namespace

extern "C" {

const char* bs_status_str(int32_t status) {
  switch (status) {
    case BS_OK: return "BS_OK";
    case BS_EINVAL: return "BS_EINVAL: invalid argument";
    case BS_ELAUNCH: return "BS_ELAUNCH: kernel launch failed";
    case BS_EWORKSPACE: return "BS_EWORKSPACE: workspace too small";
    case BS_ENODEV: return "BS_ENODEV: no usable GPU";
    default: return "unknown bs_status";
  }
}

int32_t bs_version(void) { return 100; }

int32_t bs_set_option(int32_t key, int64_t value) {
  switch (key) {
    case BS_OPT_DIRECT_PATH:
      if (value < 0 || value > 2) return BS_EINVAL;
      g_direct_path = value;
      return BS_OK;
    case BS_OPT_SIP_PATH:
      if (value < 0 || value > 4) return BS_EINVAL;
      g_sip_path = value;
      return BS_OK;
    case BS_OPT_F32_STATE:
      if (value < 0 || value > 1 + std::max(bs::compact_count(3), bs::compact_count(5)))
        return BS_EINVAL;
      g_f32_state = value;
      return BS_OK;
    case BS_OPT_EXCHANGE_WAIT_US:
      if (value < 0 || value > 10000000) return BS_EINVAL;
      bs::set_exchange_wait_us(value);
      return BS_OK;
    case BS_OPT_PART_PD_VARIANT:
    case BS_OPT_PART_TD_VARIANT: {
      const int kind = key == BS_OPT_PART_PD_VARIANT ? 5 : 3;
      if (value < 0 || value >= bs::part_variant_count(kind)) return BS_EINVAL;
      (kind == 5 ? g_pd_variant : g_td_variant) = value;
      return BS_OK;
    }
    default:
      return BS_EINVAL;
  }
}

int64_t bs_get_option(int32_t key) {
  switch (key) {
    case BS_OPT_DIRECT_PATH: return g_direct_path.load();
    case BS_OPT_PART_PD_VARIANT: return g_pd_variant.load();
    case BS_OPT_PART_TD_VARIANT: return g_td_variant.load();
    case BS_OPT_SIP_PATH: return g_sip_path.load();
    case BS_OPT_EXCHANGE_WAIT_US: return bs::exchange_wait_us();
    case BS_OPT_F32_STATE: return g_f32_state.load();
    default: return -1;
  }
}

int32_t bs_part_variant(int32_t kind, int32_t index, int32_t shape[4]) {
  if (!kind_ok(kind) || shape == nullptr) return BS_EINVAL;
  int out[4];
  if (!bs::part_variant_shape(kind, index, out)) return BS_EINVAL;
  for (int q = 0; q < 4; ++q) shape[q] = out[q];
  return BS_OK;
}

size_t bs_workspace_bytes(int32_t op, int32_t kind, int32_t dtype, int64_t n,
                          int64_t batch, int64_t ld) {
  const size_t bad = (size_t)-1;
  if (!shape_ok(n, batch, ld)) return bad;
  if (dtype != BS_F64 && dtype != BS_F32) return bad;
  const int64_t plane = n * bs::ws_ld(batch);
  if (dtype == BS_F32 && op != BS_OP_SOLVE) return bad;
  switch (op) {
    case BS_OP_FACTOR:
      return kind_ok(kind) ? 0 : bad;
    case BS_OP_SOLVE:
      if (!kind_ok(kind) || !bs::direct_supported(kind, dtype, n, ld)) return bad;
      return bs::direct_ws_bytes(kind, dtype, n, batch, ld);
    case BS_OP_SOLVE_FACTORED:
      if (!kind_ok(kind) || dtype != BS_F64) return bad;
      return g_direct_path.load() == 1 ? 0 : bs::subst_workspace_bytes(n, batch);
    case BS_OP_MNPDM: {
      const int idx = mnpdm_part_idx(n, ld);
      return idx >= 0 ? bs::part_workspace_bytes(5, idx, n, batch) : (size_t)(2 * plane) * 8;
    }
    case BS_OP_SIP: {
      // ILU(0) factors (4 planes, batch-interleaved with pitch ws_ld), then
      // one plane for the forward pass (one lane per system), the x buffers
      // and per-system state of the HB tile path, or the K x + b plane, the
      // substitution's z plane and per-system state of the exact path,
      // whichever is largest
      size_t rest = (size_t)plane * 8;
      const size_t tile = bs::sip_tile_workspace_bytes(n, batch, ld);
      const size_t exact = bs::sip_exact_supported(n, batch) ? bs::sip_exact_workspace_bytes(n, batch) : 0;
      rest = rest > tile ? rest : tile;
      rest = rest > exact ? rest : exact;
      return (size_t)(4 * plane) * 8 + rest;
    }
    case BS_OP_ADI: {
      if (!kind_ok(kind) || dtype != BS_F64) return bad;
      const int idx = g_direct_path.load() == 1 ? -1 : bs::part_adi_pick(kind, part_idx(kind), n, ld);
      return idx >= 0 ? bs::part_workspace_bytes(kind, idx, n, batch) : bad;
    }
    case BS_OP_REFINE:
      if (!kind_ok(kind) || !bs::direct_supported(kind, BS_F32, n, ld)) return bad;
      return bs::refine_workspace_bytes(kind, n, batch, ld);
    default:
      return bad;
  }
}

int32_t band_factor(int32_t kind, int32_t dtype, int64_t n, int64_t batch,
                    int64_t ld, const void* const diags[5], void* factors,
                    int32_t* info, void* stream) {
  if (!kind_ok(kind) || dtype != BS_F64 || !shape_ok(n, batch, ld)) return BS_EINVAL;
  if (!diags_ok(kind, diags, dtype) || !array_ok(factors, dtype) ||
      info == nullptr || !aligned(info, 4))
    return BS_EINVAL;
  if (!have_device()) return BS_ENODEV;
  const bs::Diags A = as_diags(kind, diags);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  double* F = static_cast<double*>(factors);
  return launched(g_direct_path.load() == 1
                      ? bs::launch_factor_lane(kind, n, batch, ld, A, F, ld, info, st)
                      : bs::launch_factor(kind, n, batch, ld, A, F, ld, info, st));
}

int32_t band_solve(int32_t kind, int32_t dtype, int64_t n, int64_t batch,
                   int64_t ld, const void* const diags[5], const void* factors,
                   const void* rhs, void* x, int32_t* info, void* workspace,
                   size_t ws_bytes, void* stream) {
  if (!kind_ok(kind) || (dtype != BS_F64 && dtype != BS_F32) || !shape_ok(n, batch, ld))
    return BS_EINVAL;
  if (!diags_ok(kind, diags, dtype) || !array_ok(rhs, dtype) ||
      !array_ok(x, dtype) || info == nullptr || !aligned(info, 4))
    return BS_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (factors != nullptr) {
    if (dtype != BS_F64 || !array_ok(factors, dtype)) return BS_EINVAL;
    const size_t need = bs_workspace_bytes(BS_OP_SOLVE_FACTORED, kind, dtype, n, batch, ld);
    if (ws_bytes < need) return BS_EWORKSPACE;
    if (need > 0 && (workspace == nullptr || !aligned(workspace, 8))) return BS_EINVAL;
    if (!have_device()) return BS_ENODEV;
    const bs::Diags A = as_diags(kind, diags);
    const double* F = static_cast<const double*>(factors);
    const double* Y = static_cast<const double*>(rhs);
    double* X = static_cast<double*>(x);
    return launched(need == 0 ? bs::launch_subst_lane(kind, n, batch, ld, A, F, Y, X, info, st)
                              : bs::launch_subst(kind, n, batch, ld, A, F, Y, X, info,
                                                 static_cast<double*>(workspace), st));
  }
  const size_t need = bs_workspace_bytes(BS_OP_SOLVE, kind, dtype, n, batch, ld);
  if (need == (size_t)-1) return BS_EINVAL;  // no kernel for this dtype and shape
  if (ws_bytes < need) return BS_EWORKSPACE;
  if (need > 0 && (workspace == nullptr || !aligned(workspace, 8))) return BS_EINVAL;
  if (!have_device()) return BS_ENODEV;
  return launched(bs::launch_direct(kind, dtype, n, batch, ld, diags, rhs, x, info,
                                    workspace, st));
}

int32_t band_solve_adi(int32_t kind, int64_t n, int64_t batch, int64_t ld, double r,
                       const double* v, double* x, int32_t* info, void* workspace,
                       size_t ws_bytes, void* stream) {
  if (!kind_ok(kind) || !shape_ok(n, batch, ld) || !(r >= 0.0) || !std::isfinite(r))
    return BS_EINVAL;
  if (!array_ok(v, BS_F64) || !array_ok(x, BS_F64) || info == nullptr || !aligned(info, 4))
    return BS_EINVAL;
  const size_t need = bs_workspace_bytes(BS_OP_ADI, kind, BS_F64, n, batch, ld);
  if (need == (size_t)-1) return BS_EINVAL;
  if (ws_bytes < need) return BS_EWORKSPACE;
  if (need > 0 && (workspace == nullptr || !aligned(workspace, 8))) return BS_EINVAL;
  if (!have_device()) return BS_ENODEV;
  const int idx = bs::part_adi_pick(kind, part_idx(kind), n, ld);
  return launched(bs::launch_part_adi(kind, idx, n, batch, ld, r, v, x, info,
                                      static_cast<double*>(workspace),
                                      static_cast<hipStream_t>(stream)));
}

int32_t band_solve_refine(int32_t kind, int64_t n, int64_t batch, int64_t ld,
                          const double* const diags[5], const double* rhs, double* x,
                          double tol, int32_t max_steps, int32_t* steps, double* relres,
                          int32_t* info, void* workspace, size_t ws_bytes, void* stream) {
  if (!kind_ok(kind) || !shape_ok(n, batch, ld)) return BS_EINVAL;
  const void* dv[5];
  for (int k = 0; k < 5; ++k) dv[k] = diags ? diags[k] : nullptr;
  if (diags == nullptr || !diags_ok(kind, dv, BS_F64) || !array_ok(rhs, BS_F64) ||
      !array_ok(x, BS_F64))
    return BS_EINVAL;
  if (steps == nullptr || !aligned(steps, 4) || !array_ok(relres, BS_F64) ||
      info == nullptr || !aligned(info, 4))
    return BS_EINVAL;
  if (!(tol > 0.0) || max_steps < 1) return BS_EINVAL;
  if ((const void*)x == (const void*)rhs) return BS_EINVAL;  // rhs is re-read every step
  const size_t need = bs_workspace_bytes(BS_OP_REFINE, kind, BS_F64, n, batch, ld);
  if (need == (size_t)-1) return BS_EINVAL;
  if (ws_bytes < need) return BS_EWORKSPACE;
  if (workspace == nullptr || !aligned(workspace, 256)) return BS_EINVAL;
  if (!have_device()) return BS_ENODEV;
  return launched(bs::launch_refine(kind, n, batch, ld, diags, rhs, x, tol, max_steps, steps,
                                    relres, info, workspace, static_cast<hipStream_t>(stream)));
}

int32_t band_solve_mnpdm(int32_t dtype, int64_t n, int64_t batch, int64_t ld,
                         const void* const cda[3], int32_t kmax,
                         const int32_t* outer_row, const void* outer_e,
                         const void* outer_b, const void* rhs, void* x,
                         int32_t* info, void* workspace, size_t ws_bytes,
                         void* stream) {
  if (dtype != BS_F64 || !shape_ok(n, batch, ld) || kmax < 0) return BS_EINVAL;
  if (cda == nullptr || !array_ok(cda[0], dtype) || !array_ok(cda[1], dtype) ||
      !array_ok(cda[2], dtype) || !array_ok(rhs, dtype) || !array_ok(x, dtype) ||
      info == nullptr || !aligned(info, 4))
    return BS_EINVAL;
  if (kmax > 0 && (outer_row == nullptr || !aligned(outer_row, 4) ||
                   !array_ok(outer_e, dtype) || !array_ok(outer_b, dtype)))
    return BS_EINVAL;
  const size_t need = bs_workspace_bytes(BS_OP_MNPDM, 5, dtype, n, batch, ld);
  if (ws_bytes < need) return BS_EWORKSPACE;
  if (need > 0 && !array_ok(workspace, dtype)) return BS_EINVAL;
  if (!have_device()) return BS_ENODEV;
  const int idx = mnpdm_part_idx(n, ld);
  if (idx >= 0) {
    const double* cd[3] = {static_cast<const double*>(cda[0]),
                           static_cast<const double*>(cda[1]),
                           static_cast<const double*>(cda[2])};
    return launched(bs::launch_part_mnpdm(
        idx, n, batch, ld, cd, kmax, outer_row, static_cast<const double*>(outer_e),
        static_cast<const double*>(outer_b), static_cast<const double*>(rhs),
        static_cast<double*>(x), info, static_cast<double*>(workspace),
        static_cast<hipStream_t>(stream)));
  }
  bs::Diags A;
  A.e = nullptr;
  A.c = static_cast<const double*>(cda[0]);
  A.d = static_cast<const double*>(cda[1]);
  A.a = static_cast<const double*>(cda[2]);
  A.b = nullptr;
  return launched(bs::launch_mnpdm_lane(
      n, batch, ld, A, kmax, outer_row, static_cast<const double*>(outer_e),
      static_cast<const double*>(outer_b), static_cast<const double*>(rhs),
      static_cast<double*>(x), info, static_cast<double*>(workspace),
      static_cast<hipStream_t>(stream)));
}

int32_t sip_solve(int32_t dtype, int64_t n, int64_t batch, int64_t ld,
                  const void* const diags[5], const void* factors,
                  const void* rhs, void* x, double tol, int32_t max_iter,
                  int32_t hb_s_L, int32_t hb_s_U, int32_t* iters,
                  double* relres, int32_t* info, void* workspace,
                  size_t ws_bytes, void* stream) {
  if (dtype != BS_F64 || !shape_ok(n, batch, ld)) return BS_EINVAL;
  if (!diags_ok(5, diags, dtype) || !array_ok(rhs, dtype) || !array_ok(x, dtype))
    return BS_EINVAL;
  if (iters == nullptr || !aligned(iters, 4) || !array_ok(relres, BS_F64) ||
      info == nullptr || !aligned(info, 4))
    return BS_EINVAL;
  if (!(tol > 0.0) || max_iter < 0) return BS_EINVAL;
  if (x == rhs) return BS_EINVAL;  // rhs is read at every step
  auto s_ok = [n](int32_t s) {
    if (s < 0 || s <= 6) return true;
    return s < 62 && (int64_t(1) << s) >= n;
  };
  if (!s_ok(hb_s_L) || !s_ok(hb_s_U)) return BS_EINVAL;
  if (factors != nullptr && !array_ok(factors, dtype)) return BS_EINVAL;
  const size_t need = bs_workspace_bytes(BS_OP_SIP, 5, dtype, n, batch, ld);
  if (ws_bytes < need) return BS_EWORKSPACE;
  if (!array_ok(workspace, dtype)) return BS_EINVAL;
  if (!have_device()) return BS_ENODEV;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const bs::Diags A = as_diags(5, diags);
  double* ws = static_cast<double*>(workspace);
  const int64_t lw = bs::ws_ld(batch);
  const double* F = static_cast<const double*>(factors);
  int64_t fld = ld;  // pitch of caller-provided factors (band_factor output)
  const bool own = F == nullptr;
  if (own) {
    // ILU(0) into the first 4 workspace planes (pitch lw)
    fld = lw;
    const hipError_t fe = g_direct_path.load() == 1
                              ? bs::launch_factor_lane(5, n, batch, ld, A, ws, fld, info, st)
                              : bs::launch_factor(5, n, batch, ld, A, ws, fld, info, st);
    if (fe != hipSuccess)
      return BS_ELAUNCH;
    F = ws;
  }
  double* rest = ws + 4 * n * lw;  // 256-byte aligned: lw is a multiple of 64
  const int64_t path = g_sip_path.load();
  // HB with 2^s >= n is the exact inverse: both factors exact is Algorithm 1
  // as printed
  auto exact = [n](int32_t s) { return s < 0 || (s < 62 && (int64_t(1) << s) >= n); };
  if (path != 1 && exact(hb_s_L) && exact(hb_s_U) && bs::sip_exact_supported(n, batch))
    return launched(bs::launch_sip_exact(n, batch, ld, A, F, fld,
                                         static_cast<const double*>(rhs),
                                         static_cast<double*>(x), tol, max_iter, iters, relres,
                                         info, rest, st));
  if (path != 1 && bs::sip_tile_supported(n, hb_s_L, hb_s_U))
    return launched(bs::launch_sip_tile(n, batch, ld, A, F, fld, own,
                                        static_cast<const double*>(rhs),
                                        static_cast<double*>(x), tol, max_iter, hb_s_L,
                                        hb_s_U, iters, relres, info, rest,
                                        path == 3 ? 1 : (path == 4 ? 2 : 3), st));
  return launched(bs::launch_sip_lane(n, batch, ld, A, F, fld,
                                      static_cast<const double*>(rhs),
                                      static_cast<double*>(x), tol, max_iter,
                                      hb_s_L, hb_s_U, iters, relres, info, rest, st));
}

static bool layout_ok(int64_t n, int64_t batch, int64_t ld, int64_t pitch, const void* a,
                      const void* b) {
  constexpr int64_t kMax = int64_t(1) << 26;
  return n >= 1 && batch >= 1 && n < kMax && batch < kMax && ld >= batch && pitch >= n &&
         a != nullptr && b != nullptr && aligned(a, 8) && aligned(b, 8);
}

int32_t bs_pack_interleave(int64_t n, int64_t batch, const double* src, int64_t src_pitch,
                           double* dst, int64_t ld, void* stream) {
  if (!layout_ok(n, batch, ld, src_pitch, src, dst)) return BS_EINVAL;
  if (!have_device()) return BS_ENODEV;
  // src is [batch][src_pitch]: R = batch rows of n columns
  return launched(bs::launch_transpose64(batch, n, src, src_pitch, dst, ld,
                                         static_cast<hipStream_t>(stream)));
}

int32_t bs_unpack_interleave(int64_t n, int64_t batch, const double* src, int64_t ld,
                             double* dst, int64_t dst_pitch, void* stream) {
  if (!layout_ok(n, batch, ld, dst_pitch, src, dst)) return BS_EINVAL;
  if (!have_device()) return BS_ENODEV;
  return launched(bs::launch_transpose64(n, batch, src, ld, dst, dst_pitch,
                                         static_cast<hipStream_t>(stream)));
}

int32_t bs_stream_probe(int64_t count, int32_t nin, const double* const in[6], double* out,
                        void* stream) {
  if (count < 2 || count % 2 != 0 || nin < 1 || nin > 6 || in == nullptr || out == nullptr ||
      !aligned(out, 16))
    return BS_EINVAL;
  for (int k = 0; k < nin; ++k)
    if (in[k] == nullptr || !aligned(in[k], 16)) return BS_EINVAL;
  if (!have_device()) return BS_ENODEV;
  return launched(bs::launch_stream_probe(count, nin, in, out, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
