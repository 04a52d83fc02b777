// stream_probe.hip -- the HBM ceiling of the solvers' traffic pattern: a plain
// streaming kernel that reads `nin` arrays once and writes one, with no
// dependence between elements.  The rate it reaches is the practical
// bandwidth against which the solver kernels' algorithmic rates are judged.
#include "bs_internal.h"

namespace bs {
namespace {

constexpr int kBlock = 256;
typedef double dbl2 __attribute__((ext_vector_type(2)));

struct In6 {
  const double* p[6];
};

// 16-byte loads and stores: out[2i..2i+1] = sum_k in_k[2i..2i+1].
template <int NIN>
__global__ __launch_bounds__(kBlock) void stream_kernel(int64_t pairs, In6 in,
                                                        double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < pairs; q += stride) {
    dbl2 acc = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(in.p[0]) + q);
#pragma unroll
    for (int k = 1; k < NIN; ++k)
      acc += __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(in.p[k]) + q);
    __builtin_nontemporal_store(acc, reinterpret_cast<dbl2*>(out) + q);
  }
}

}  // namespace

hipError_t launch_stream_probe(int64_t count, int nin, const double* const* in, double* out,
                               hipStream_t st) {
  In6 a{};
  for (int k = 0; k < nin; ++k) a.p[k] = in[k];
  const int64_t pairs = count / 2;
  int64_t blocks = (pairs + kBlock - 1) / kBlock;
  if (blocks > 16384) blocks = 16384;  // grid-stride beyond 64 blocks per CU
  if (blocks < 1) blocks = 1;
  switch (nin) {
#define BS_SP(K) \
  case K:        \
    hipLaunchKernelGGL(stream_kernel<K>, dim3((unsigned)blocks), dim3(kBlock), 0, st, pairs, a, out); \
    break;
    BS_SP(1) BS_SP(2) BS_SP(3) BS_SP(4) BS_SP(5) BS_SP(6)
#undef BS_SP
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace bs
