// ga_children_f.hip -- children kernels of orders 60 and 64 (the templates are in
// ga_children.h; the orders are spread over several files so that they
// compile in parallel).
#include "ga_children.h"

namespace ga {

GA_DEFINE_ORDER(60) GA_DEFINE_ORDER(64)

}  // namespace ga
