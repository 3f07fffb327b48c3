// ga_children_k.hip -- children kernels of orders 100 and 104 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(100) GA_DEFINE_ORDER(104)

}  // namespace ga
