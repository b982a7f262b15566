// Instantiation unit of the k-best bound kernel for one norm (all d,
// monotone counts and list lengths).
#include "bounds_topk.hpp"

namespace lip {

TopkLaunch topk_linf(int d, int dm, int kl) { return topk_table_kl<3>(d, dm, kl); }

}  // namespace lip
