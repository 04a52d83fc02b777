// direct_part.hip -- partitioned (multi-lane per system) direct solvers.
#include "bs_internal.h"

namespace bs {

bool part_supported(int, int64_t, int64_t) { return false; }

hipError_t launch_part(int, int64_t, int64_t, int64_t, Diags, const double*,
                       double*, int32_t*, hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace bs
