// Instantiation unit of the k-best bound kernel for one norm (all d,
// monotone counts and list lengths).
#include "bounds_topk.hpp"

namespace lip {

TopkLaunch topk_l1(int d, int dm, int kl) { return topk_table_kl<1>(d, dm, kl); }

}  // namespace lip
