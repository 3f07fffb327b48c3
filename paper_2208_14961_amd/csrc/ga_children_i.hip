// ga_children_i.hip -- children kernels of orders 84 and 88 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(84) GA_DEFINE_ORDER(88)

}  // namespace ga
