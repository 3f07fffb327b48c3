// ga_tuning.hip -- the tuning table's lookup (host only).
#include "ga_internal.h"
#include "ga_tuned.h"

namespace ga {

// Gram products of the standalone fitness on the matrix cores (1) or by
// popcount (0), per order 4, 8, .., 128.
static const uint8_t kMfmaFitness[32] = {
    0, 0, 0, 0, 0, 0, 0, 0,  // orders 4..32: one-word columns, popcount only
    0, 0, 0, 0, 0, 0, 0, 0,  // orders 36..64
    0, 0, 0, 0, 0, 0, 0, 0,  // orders 68..96
    0, 0, 0, 0, 0, 0, 0, 0,  // orders 100..128
};

bool use_mfma(const ga_config* c) {
  const uint32_t gram = c->flags & GA_GRAM_MASK;
  if (gram == GA_GRAM_MFMA) return true;
  if (gram == GA_GRAM_PACKED || c->m < kMfmaMinOrder) return false;
  return kMfmaFitness[c->m / 4 - 1] != 0;
}

uint32_t tuned_lanes(uint32_t m, uint64_t children) {
  const uint32_t row = m / 4 - 1;
  int j = 0;
  while (j + 1 < kTuneSizes && children > kTuneMaxChildren[j]) ++j;
  const uint32_t lanes = kTunedLanes[row][j];
  return lanes_allowed(m, lanes) ? lanes : (m <= 32 ? 4u : 8u);
}

}  // namespace ga
