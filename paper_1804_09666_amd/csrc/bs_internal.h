// bs_internal.h -- launchers shared between the ABI layer and the kernels of
// libbandsolve.  Not part of the public ABI (see include/bandsolve.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bs {

// Leading dimension used for workspace arrays: batch rounded up to 64 so that
// one row of a wave's 64 systems is one aligned 512-byte segment.
inline int64_t ws_ld(int64_t batch) { return (batch + 63) / 64 * 64; }

struct Diags {
  const double* e;
  const double* c;
  const double* d;
  const double* a;
  const double* b;
};

// ---- direct solvers, one lane per system (direct_lane.hip) --------------
hipError_t launch_npdm_lane(int64_t n, int64_t batch, int64_t ld, Diags A,
                            const double* y, double* x, int32_t* info,
                            double* ws, hipStream_t st);
hipError_t launch_ntdm_lane(int64_t n, int64_t batch, int64_t ld, Diags A,
                            const double* y, double* x, int32_t* info,
                            double* ws, hipStream_t st);
hipError_t launch_mnpdm_lane(int64_t n, int64_t batch, int64_t ld, Diags A,
                             int32_t kmax, const int32_t* orow,
                             const double* oe, const double* ob,
                             const double* y, double* x, int32_t* info,
                             double* ws, hipStream_t st);
// factors are written with pitch fld (array k at factors + k*n*fld).
// launch_factor splits the rows of a system over lanes where the batch is
// too small to fill the GPU (bitwise the same factors and info);
// launch_factor_lane keeps one lane per system.
hipError_t launch_factor(int kind, int64_t n, int64_t batch, int64_t ld, Diags A,
                         double* factors, int64_t fld, int32_t* info, hipStream_t st);
hipError_t launch_factor_lane(int kind, int64_t n, int64_t batch, int64_t ld,
                              Diags A, double* factors, int64_t fld,
                              int32_t* info, hipStream_t st);
hipError_t launch_subst_lane(int kind, int64_t n, int64_t batch, int64_t ld,
                             Diags A, const double* factors, const double* y,
                             double* x, int32_t* info, hipStream_t st);
// Substitution with the rows split over lanes where the batch is small
// (bitwise the one-lane result); z goes through ws, subst_workspace_bytes
// long (0: one lane per system, ws unused).
size_t subst_workspace_bytes(int64_t n, int64_t batch);
// Chunks per system of the split substitution (1: one lane per system).
int64_t subst_chunks(int64_t n, int64_t batch);
// The split substitution (subst_chunks > 1) of the systems with active[s] != 0
// (all when NULL): rhs y with pitch yl, factors with pitch fld, x with pitch
// ld; z and the proof flags in ws (subst_workspace_bytes); every launch
// returns at once when done != NULL and *done != 0; info (nullable) = 0.
hipError_t launch_subst_masked(int kind, int64_t n, int64_t batch, int64_t ld, Diags A,
                               const double* factors, int64_t fld, const double* y, int64_t yl,
                               double* x, int32_t* info, double* ws, const int32_t* active,
                               const int32_t* done, hipStream_t st);
hipError_t launch_subst(int kind, int64_t n, int64_t batch, int64_t ld, Diags A,
                        const double* factors, const double* y, double* x, int32_t* info,
                        double* ws, hipStream_t st);

// ---- direct solvers, rows of a system split over lanes (direct_part.hip) --
// Variant idx of a kind: M rows per lane, PW lanes per system in a block
// (one tile of M*PW rows), G systems per block, up to TMAX tiles per system,
// all in one launch.  dtype 0: FP64 storage, 1: FP32 storage; arithmetic is
// FP64 in both.
int part_variant_count(int kind);
// Longest wait (microseconds) of a split-kernel tile for the other tiles of
// its system before it gives up (info = -4); process-wide.
void set_exchange_wait_us(int64_t us);
int64_t exchange_wait_us();
bool part_variant_shape(int kind, int idx, int out[4]);
// The configured variant if it handles (n, ld, dtype), else the first one
// that does; -1 if none.
int part_pick(int kind, int idx, int64_t n, int64_t ld, int dtype);
size_t part_workspace_bytes(int kind, int idx, int64_t n, int64_t batch);
// Leading bytes of that workspace that must be zero before a launch (the
// meeting counters; 0 when a system fits one tile).
size_t part_counter_bytes(int kind, int idx, int64_t n, int64_t batch);
// skip (nullable device flag): when *skip != 0 at launch the kernels return
// at once (a refinement loop that has converged).
hipError_t launch_part(int kind, int idx, int dtype, int64_t n, int64_t batch, int64_t ld,
                       const void* const dg[5], const void* y, void* x, int32_t* info,
                       double* ws, hipStream_t st, const int32_t* skip = nullptr);
// FP32 storage with the compact chunk state (FP32 per-row state and backward
// substitution, FP64 forward recurrences): variant idx of a kind (as
// part_pick: the preferred one if it covers n, else the first that does, -1
// if none), its workspace, leading counter bytes and launch.
int compact_count(int kind);
int compact_pick(int kind, int idx, int64_t n, int64_t ld, int dtype = 1);
size_t compact_workspace_bytes(int kind, int idx, int64_t n, int64_t batch);
size_t compact_counter_bytes(int kind, int idx, int64_t n, int64_t batch);
hipError_t launch_compact(int kind, int idx, int64_t n, int64_t batch, int64_t ld,
                          const void* const dg[5], const void* y, void* x, int32_t* info,
                          double* ws, hipStream_t st, const int32_t* skip = nullptr);
// The compact-state kernels on FP64 storage (FP64 matrix, right-hand side
// and x; FP32 per-row state, so x has the compact state's FP32-level error):
// the refinement's solves.  acc: x += the solution instead of x = (the
// variant and workspace as compact_pick / compact_workspace_bytes); act
// (nullable): systems with act[s] == 0 are not touched (x, info).
hipError_t launch_compact_f64(int kind, int idx, int64_t n, int64_t batch, int64_t ld,
                              const double* const dg[5], const double* y, double* x,
                              int32_t* info, double* ws, hipStream_t st, const int32_t* skip,
                              bool acc, const int32_t* act);
// MNPDM (outer diagonals as a per-system list) on the split kernels: the
// variant to use for (n, ld) (-1 if none) and its launch; the workspace is
// part_workspace_bytes(5, idx, n, batch).
int part_mnpdm_pick(int idx, int64_t n, int64_t ld);
hipError_t launch_part_mnpdm(int idx, int64_t n, int64_t batch, int64_t ld,
                             const double* const cda[3], int32_t kmax, const int32_t* orow,
                             const double* oe, const double* ob, const double* y, double* x,
                             int32_t* info, double* ws, hipStream_t st);
// The ADI sweep assembled inside the split kernels (first two variants):
// the variant for (n, ld) or -1, and its launch.  ws as part_workspace_bytes.
int part_adi_pick(int kind, int idx, int64_t n, int64_t ld);
hipError_t launch_part_adi(int kind, int idx, int64_t n, int64_t batch, int64_t ld, double r,
                           const double* v, double* x, int32_t* info, double* ws,
                           hipStream_t st);
// Any length: three launches (tile maps, per-system reduction, finish).
bool long_supported(int64_t n, int64_t ld, int dtype);
size_t long_workspace_bytes(int kind, int64_t n, int64_t batch);
hipError_t launch_long_path(int kind, int dtype, int64_t n, int64_t batch, int64_t ld,
                            const void* const dg[5], const void* y, void* x, int32_t* info,
                            double* ws, hipStream_t st, const int32_t* skip = nullptr);

// ---- mixed-precision refinement (refine.hip) ------------------------------
// BS_OPT_F32_STATE != 0 (abi.hip): the compact chunk state is in use.
bool f32_compact_state();
size_t refine_workspace_bytes(int kind, int64_t n, int64_t batch, int64_t ld);
hipError_t launch_refine(int kind, int64_t n, int64_t batch, int64_t ld, const double* const dg[5],
                         const double* rhs, double* x, double tol, int32_t max_steps,
                         int32_t* steps, double* relres, int32_t* info, void* ws,
                         hipStream_t st);

// Fused FP32/FP64 direct solve selection shared by band_solve and refinement:
// bytes of workspace and the launch for (kind, dtype, n, batch, ld).
size_t direct_ws_bytes(int kind, int dtype, int64_t n, int64_t batch, int64_t ld);
hipError_t launch_direct(int kind, int dtype, int64_t n, int64_t batch, int64_t ld,
                         const void* const dg[5], const void* y, void* x, int32_t* info,
                         void* ws, hipStream_t st, const int32_t* skip = nullptr);
// false if no kernel handles this (FP32 storage needs the split or long path).
bool direct_supported(int kind, int dtype, int64_t n, int64_t ld);
// Leading bytes of the fused solve's workspace that must be zero at launch.
size_t direct_counter_bytes(int kind, int dtype, int64_t n, int64_t batch, int64_t ld);

// ---- SIP (sip_lane.hip) --------------------------------------------------
hipError_t launch_sip_lane(int64_t n, int64_t batch, int64_t ld, Diags A,
                           const double* factors, int64_t fld,
                           const double* y, double* x,
                           double tol, int32_t max_iter, int32_t sL,
                           int32_t sU, int32_t* iters, double* relres,
                           int32_t* info, double* v_ws, hipStream_t st);

// ---- SIP as Algorithm 1 (exact substitutions), rows split (sip_exact.hip) --
// Row-parallel residual and K x + b, the stopping test in the last block,
// the split substitution; bitwise the one-lane kernel.  Needs
// subst_chunks(n, batch) > 1.
bool sip_exact_supported(int64_t n, int64_t batch);
size_t sip_exact_workspace_bytes(int64_t n, int64_t batch);
hipError_t launch_sip_exact(int64_t n, int64_t batch, int64_t ld, Diags A, const double* factors,
                            int64_t fld, const double* y, double* x, double tol,
                            int32_t max_iter, int32_t* iters, double* relres, int32_t* info,
                            void* ws, hipStream_t st);

// ---- SIP with HB steps, rows split over lanes (sip_tile.hip) -------------
// Both s_L, s_U >= 0, HB not exact (2^s <= n) and halos that leave a tile
// core of at least 64 rows.
bool sip_tile_supported(int64_t n, int32_t sL, int32_t sU);
size_t sip_tile_workspace_bytes(int64_t n, int64_t batch, int64_t ld);
// own_factors: the factors were just computed by launch_factor_lane, whose
// info marks systems that cannot step.  steps_per_launch: 2 takes two steps
// per launch where the halos allow it, 1 one step per launch.
hipError_t launch_sip_tile(int64_t n, int64_t batch, int64_t ld, Diags A, const double* factors,
                           int64_t fld, bool own_factors, const double* y, double* x, double tol,
                           int32_t max_iter, int32_t sL, int32_t sU, int32_t* iters,
                           double* relres, int32_t* info, void* ws, int steps_per_launch,
                           hipStream_t st);

// ---- layout conversion (layout.hip) -------------------------------------
// dst[c * dpitch + r] = src[r * spitch + c] for r < R, c < C (R, C < 2^21 * 32).
hipError_t launch_transpose64(int64_t R, int64_t C, const double* src, int64_t spitch,
                              double* dst, int64_t dpitch, hipStream_t st);

// ---- measurement (stream_probe.hip) -------------------------------------
// out = in_0 + ... + in_{nin-1} elementwise (count even, 16-byte aligned).
hipError_t launch_stream_probe(int64_t count, int nin, const double* const* in, double* out,
                               hipStream_t st);

}  // namespace bs
