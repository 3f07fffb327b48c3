// ga_children_m.hip -- children kernels of orders 116 and 120 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(116) GA_DEFINE_ORDER(120)

}  // namespace ga
