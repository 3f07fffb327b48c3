// ga_children.hip -- dispatch of the children launches to the per-order
// entry points (ga_children_a..n.hip).
#include "ga_children.h"

namespace ga {

hipError_t launch_children(const PopDesc* descs_dev, const uint32_t* block_pop,
                           uint32_t total_blocks, uint32_t m, uint32_t lanes,
                           uint32_t node, hipStream_t s) {
  if (total_blocks == 0) return hipSuccess;
  switch (m) {
#define GA_MULTI_CASE(MM)                                                      \
  case MM:                                                                     \
    return launch_children_multi_m##MM(descs_dev, block_pop, total_blocks,     \
                                       lanes, node, s);
    GA_FOR_EACH_ORDER(GA_MULTI_CASE)
#undef GA_MULTI_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_children_one(const PopDesc& d, uint32_t node, hipStream_t s) {
  if (d.nblocks == 0) return hipSuccess;
  switch (d.m) {
#define GA_ONE_CASE(MM) \
  case MM:              \
    return launch_children_one_m##MM(d, node, s);
    GA_FOR_EACH_ORDER(GA_ONE_CASE)
#undef GA_ONE_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace ga
