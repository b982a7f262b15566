// Instantiation unit of the fused bound kernel for one norm (all d, all
// monotone-coordinate counts).
#include "bounds_fwd.hpp"

namespace lip {

FwdLauncher fwd_launcher_linf(int d, int dm) { return fwd_table<kNormLinf>(d, dm); }

}  // namespace lip
