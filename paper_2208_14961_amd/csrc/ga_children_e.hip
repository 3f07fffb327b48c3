// ga_children_e.hip -- children kernels of orders 52 and 56 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(52) GA_DEFINE_ORDER(56)

}  // namespace ga
