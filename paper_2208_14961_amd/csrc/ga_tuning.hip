// ga_tuning.hip -- the tuning table's lookup (host only).
#include "ga_internal.h"
#include "ga_tuned.h"

namespace ga {

// Gram products of the standalone fitness on the matrix cores (1) or by
// popcount (0), per order 4, 8, .., 128.  Measured with ga_fitness_repeat
// (SQ, n = 40,000, about 2 ms per launch, one MI355X), 10^9 evaluations/s
// popcount vs matrix cores:
//   m = 36: 1.74 vs 2.71
//   m = 40: 1.44 vs 2.76
//   m = 44: 1.12 vs 2.73
//   m = 48: 2.14 vs 2.75
//   m = 52: 1.51 vs 1.99
//   m = 56: 1.48 vs 1.98
//   m = 60: 1.14 vs 1.97
//   m = 64: 1.20 vs 2.00
//   m = 68: 0.76 vs 1.13
//   m = 72: 0.75 vs 1.13
//   m = 76: 0.62 vs 1.13
//   m = 80: 0.57 vs 1.13
//   m = 84: 0.51 vs 0.87
//   m = 88: 0.50 vs 0.87
//   m = 92: 0.43 vs 0.87
//   m = 96: 0.40 vs 0.88
//   m = 100: 0.37 vs 0.70
//   m = 104: 0.35 vs 0.69
//   m = 108: 0.31 vs 0.70
//   m = 112: 0.30 vs 0.69
//   m = 116: 0.28 vs 0.57
//   m = 120: 0.27 vs 0.57
//   m = 124: 0.24 vs 0.57
//   m = 128: 0.26 vs 0.57
static const uint8_t kMfmaFitness[32] = {
    0, 0, 0, 0, 0, 0, 0, 0,  // orders 4..32: one-word columns, popcount only
    1, 1, 1, 1, 1, 1, 1, 1,  // orders 36..64
    1, 1, 1, 1, 1, 1, 1, 1,  // orders 68..96
    1, 1, 1, 1, 1, 1, 1, 1,  // orders 100..128
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
