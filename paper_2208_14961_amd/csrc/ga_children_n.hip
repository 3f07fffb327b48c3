// ga_children_n.hip -- children kernels of orders 124 and 128 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(124) GA_DEFINE_ORDER(128)

}  // namespace ga
