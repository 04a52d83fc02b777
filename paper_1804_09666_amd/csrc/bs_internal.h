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
// factors are written with pitch fld (array k at factors + k*n*fld)
hipError_t launch_factor_lane(int kind, int64_t n, int64_t batch, int64_t ld,
                              Diags A, double* factors, int64_t fld,
                              int32_t* info, hipStream_t st);
hipError_t launch_subst_lane(int kind, int64_t n, int64_t batch, int64_t ld,
                             Diags A, const double* factors, const double* y,
                             double* x, int32_t* info, hipStream_t st);

// ---- direct solvers, rows of a system split over lanes (direct_part.hip) --
// Variant idx of a kind: M rows per lane, PW lanes per system in a block
// (one tile of M*PW rows), G systems per block, up to TMAX tiles per system.
int part_variant_count(int kind);
bool part_variant_shape(int kind, int idx, int out[4]);
bool part_supported(int kind, int idx, int64_t n, int64_t batch, int64_t ld);
size_t part_workspace_bytes(int kind, int idx, int64_t n, int64_t batch);
hipError_t launch_part(int kind, int idx, int64_t n, int64_t batch, int64_t ld,
                       Diags A, const double* y, double* x, int32_t* info,
                       double* ws, hipStream_t st);

// ---- SIP (sip_lane.hip) --------------------------------------------------
hipError_t launch_sip_lane(int64_t n, int64_t batch, int64_t ld, Diags A,
                           const double* factors, int64_t fld,
                           const double* y, double* x,
                           double tol, int32_t max_iter, int32_t sL,
                           int32_t sU, int32_t* iters, double* relres,
                           int32_t* info, double* v_ws, hipStream_t st);

}  // namespace bs
