// ga_children_l.hip -- children kernels of orders 108 and 112 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(108) GA_DEFINE_ORDER(112)

}  // namespace ga
