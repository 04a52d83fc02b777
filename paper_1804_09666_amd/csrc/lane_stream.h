// lane_stream.h -- row streaming with register prefetch for the kernels in
// which one lane walks the rows of one system.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bs {

// When one lane walks the rows of one system its recurrence is serial, and
// with few systems (one wave per 64 of them) a load issued when its row comes
// up would expose the whole memory latency on every row.  stream_rows walks rows 0..n-1 (or n-1..0)
// with the loads of row k + PF issued while row k is processed: a ring of
// PF rows in registers, rotated by a fully unrolled inner loop so that every
// ring slot is a fixed register.  fetch(slot, i) loads row i into the slot
// (rows past the end re-load the last row: a valid address, never used);
// use(slot, i) consumes it.  The loop bounds are uniform across the wave and
// nothing inside exits early, so no ring value has to be merged (and waited
// for) at a control-flow join.
template <int PF, bool DESC, typename Fetch, typename Use>
__device__ __forceinline__ void stream_rows(int64_t n, Fetch&& fetch, Use&& use) {
  auto row_of = [n](int64_t k) { return DESC ? n - 1 - k : k; };
  auto clamp = [n](int64_t k) { return k < n ? k : n - 1; };
  const int64_t nfull = n / PF * PF;
#pragma unroll
  for (int q = 0; q < PF; ++q) fetch(q, row_of(clamp(q)));
  for (int64_t k0 = 0; k0 < nfull; k0 += PF) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      use(q, row_of(k0 + q));
      fetch(q, row_of(clamp(k0 + q + PF)));
    }
  }
  for (int64_t k = nfull; k < n; ++k) {  // the last rows are already in the ring
#pragma unroll
    for (int q = 0; q < PF; ++q)
      if (q == k - nfull) use(q, row_of(k));
  }
}

}  // namespace bs
