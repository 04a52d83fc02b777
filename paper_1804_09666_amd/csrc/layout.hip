// layout.hip -- conversions between system-contiguous lines and the batch-
// interleaved layout every solver reads (element (row i, system s) at
// p[i*ld + s]).  The lines of an ADI sweep along the fast axis of a row-major
// grid are system-contiguous; the sweep along the other axis is already
// interleaved, so alternating sweeps convert once per step.  A 32 x 32 tile
// goes through LDS so that both the reads and the writes are 256-byte rows.
#include "bs_internal.h"

namespace bs {
namespace {

constexpr int kT = 32;

// dst[c * dpitch + r] = src[r * spitch + c] for r < R, c < C.
__global__ __launch_bounds__(256) void transpose64_kernel(int64_t R, int64_t C,
                                                          const double* __restrict__ src,
                                                          int64_t spitch, double* __restrict__ dst,
                                                          int64_t dpitch) {
  __shared__ double tile[kT][kT + 1];
  const int64_t r0 = (int64_t)blockIdx.y * kT, c0 = (int64_t)blockIdx.x * kT;
  const int tx = threadIdx.x & (kT - 1), ty = threadIdx.x / kT;  // 32 x 8
  for (int k = ty; k < kT; k += 8)
    if (r0 + k < R && c0 + tx < C) tile[k][tx] = src[(r0 + k) * spitch + c0 + tx];
  __syncthreads();
  for (int k = ty; k < kT; k += 8)
    if (c0 + k < C && r0 + tx < R) dst[(c0 + k) * dpitch + r0 + tx] = tile[tx][k];
}

}  // namespace

hipError_t launch_transpose64(int64_t R, int64_t C, const double* src, int64_t spitch,
                              double* dst, int64_t dpitch, hipStream_t st) {
  const dim3 grid((unsigned)((C + kT - 1) / kT), (unsigned)((R + kT - 1) / kT));
  hipLaunchKernelGGL(transpose64_kernel, grid, dim3(256), 0, st, R, C, src, spitch, dst, dpitch);
  return hipGetLastError();
}

}  // namespace bs
