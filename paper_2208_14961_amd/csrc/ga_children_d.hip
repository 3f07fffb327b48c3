// ga_children_d.hip -- children kernels of orders 44 and 48 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(44) GA_DEFINE_ORDER(48)

}  // namespace ga
