// ga_tuning.hip -- the tuning table's lookup (host only).
#include "ga_internal.h"
#include "ga_tuned.h"

namespace ga {

uint32_t tuned_lanes(uint32_t m, uint64_t children) {
  const uint32_t row = m / 4 - 1;
  int j = 0;
  while (j + 1 < kTuneSizes && children > kTuneMaxChildren[j]) ++j;
  const uint32_t lanes = kTunedLanes[row][j];
  return lanes_allowed(m, lanes) ? lanes : (m <= 32 ? 4u : 8u);
}

}  // namespace ga
