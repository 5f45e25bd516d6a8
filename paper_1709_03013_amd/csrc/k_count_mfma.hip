// k_count_mfma.hip -- interval counting as an int8 MFMA contraction.
#include "cs_internal.h"

namespace cs {
hipError_t launch_count_mfma(const uint64_t* bits, int64_t N, int64_t W, int kmax,
                             uint64_t* rb_stats, hipStream_t st) {
  (void)bits; (void)N; (void)W; (void)kmax; (void)rb_stats; (void)st;
  return hipErrorNotSupported;
}
}  // namespace cs
