// Instantiation unit of the fused bound kernel for one norm (all d, all
// monotone-coordinate counts).
#include "bounds_fwd.hpp"

namespace lip {

FwdLauncher fwd_launcher_l2(int d, int dm) { return fwd_table<kNormL2>(d, dm); }

}  // namespace lip
