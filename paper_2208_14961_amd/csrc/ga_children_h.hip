// ga_children_h.hip -- children kernels of orders 76 and 80 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(76) GA_DEFINE_ORDER(80)

}  // namespace ga
