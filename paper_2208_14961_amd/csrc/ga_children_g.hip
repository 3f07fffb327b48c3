// ga_children_g.hip -- children kernels of orders 68 and 72 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(68) GA_DEFINE_ORDER(72)

}  // namespace ga
