// noalloc.hip -- band_solve_noalloc: the fused band_solve with its scratch
// memory (the split kernels' meeting counters, tile maps and redo planes, or
// the one-lane kernels' alpha / beta planes) in a static device array instead
// of a caller workspace, for callers that cannot allocate.
#include <stdint.h>

#include <mutex>

#include "bandsolve.h"
#include "bs_internal.h"

namespace {

// The scratch of every call on a device: the array is zero when the module
// is loaded, and each device holds its own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[BS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of the current device's copy (looked up once per device).
void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lock(g_mutex);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

// Zero the first `words` 32-bit words (a fill kernel, not a memset node: the
// call may be captured in a graph).
__global__ __launch_bounds__(256) void zero_words(uint32_t* __restrict__ p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * 256)
    p[i] = 0u;
}

bool shape_ok(int64_t n, int64_t batch, int64_t ld) {
  return n >= 1 && batch >= 1 && ld >= batch && n < (int64_t(1) << 31) - 1 &&
         batch < (int64_t(1) << 31) && ld <= (int64_t(1) << 50) / n;
}

bool array_ok(const void* p, int32_t dtype) {
  return p != nullptr && reinterpret_cast<uintptr_t>(p) % (dtype == BS_F32 ? 4 : 8) == 0;
}

}  // namespace

extern "C" int32_t band_solve_noalloc(int32_t kind, int32_t dtype, int64_t n, int64_t batch,
                                      int64_t ld, const void* const diags[5], const void* rhs,
                                      void* x, int32_t* info, void* stream) {
  if ((kind != 3 && kind != 5) || (dtype != BS_F64 && dtype != BS_F32) ||
      !shape_ok(n, batch, ld) || diags == nullptr)
    return BS_EINVAL;
  for (int k = 0; k < 5; ++k)
    if ((kind == 5 || (k >= 1 && k <= 3)) && !array_ok(diags[k], dtype)) return BS_EINVAL;
  if (!array_ok(rhs, dtype) || !array_ok(x, dtype) || info == nullptr ||
      reinterpret_cast<uintptr_t>(info) % 4 != 0)
    return BS_EINVAL;
  const size_t need = bs_workspace_bytes(BS_OP_SOLVE, kind, dtype, n, batch, ld);
  if (need == (size_t)-1) return BS_EINVAL;
  if (need > (size_t)BS_NOALLOC_SCRATCH_BYTES) return BS_EWORKSPACE;
  int dev = -1, count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1 || hipGetDevice(&dev) != hipSuccess ||
      dev < 0 || dev >= kMaxDevices)
    return BS_ENODEV;
  void* ws = scratch_ptr(dev);
  if (ws == nullptr) return BS_ELAUNCH;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t zero = bs::direct_counter_bytes(kind, dtype, n, batch, ld);
  if (zero > 0) {
    const int64_t words = (int64_t)(zero / 4);
    const int64_t blocks = (words + 255) / 256;
    hipLaunchKernelGGL(zero_words, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0,
                       st, static_cast<uint32_t*>(ws), words);
    if (hipGetLastError() != hipSuccess) return BS_ELAUNCH;
  }
  return bs::launch_direct(kind, dtype, n, batch, ld, diags, rhs, x, info, ws, st) == hipSuccess
             ? BS_OK
             : BS_ELAUNCH;
}
