// ga_children_j.hip -- children kernels of orders 92 and 96 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(92) GA_DEFINE_ORDER(96)

}  // namespace ga
