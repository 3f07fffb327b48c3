// ga_children_b.hip -- children kernels of orders 20..32 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(20) GA_DEFINE_ORDER(24) GA_DEFINE_ORDER(28) GA_DEFINE_ORDER(32)

}  // namespace ga
