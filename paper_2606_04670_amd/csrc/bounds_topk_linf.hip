// Instantiation unit of the k-best bound kernel for one norm (all d and
// monotone counts).
#include "bounds_topk.hpp"

namespace lip {

TopkLaunch topk_linf(int d, int dm) { return topk_table<3>(d, dm); }

}  // namespace lip
