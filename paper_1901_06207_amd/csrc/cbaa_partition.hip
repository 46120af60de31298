// Partitioned update path (LDS tiles). Not enabled yet: callers fall back to
// direct atomics.
#include "cbaa_internal.hpp"

namespace cbaa {

bool partitioned_supported(const Dims&) { return false; }
uint64_t partitioned_scratch_bytes(const Dims&, uint64_t, int) { return 0; }
uint64_t partitioned_min_scratch_bytes(const Dims&, int) { return 0; }
int launch_update_partitioned(const Dims& d, uint64_t* c0, uint64_t* c1, const uint32_t* pairs,
                              uint64_t n, int side, void*, uint64_t, hipStream_t s) {
  return launch_update_direct(d, c0, c1, pairs, n, side, s);
}

}  // namespace cbaa
