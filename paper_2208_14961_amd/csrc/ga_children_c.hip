// ga_children_c.hip -- children kernels of orders 36 and 40 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(36) GA_DEFINE_ORDER(40)

}  // namespace ga
