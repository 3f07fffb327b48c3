// ga_children_a.hip -- children kernels of orders 4..16 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(4) GA_DEFINE_ORDER(8) GA_DEFINE_ORDER(12) GA_DEFINE_ORDER(16)

}  // namespace ga
