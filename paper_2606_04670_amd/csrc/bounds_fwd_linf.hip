// Instantiation unit of the fused bound kernels (plain and batched) for one
// norm (all d, all monotone-coordinate counts).
#include "bounds_fwd.hpp"

namespace lip {

FwdLaunchers fwd_launchers_linf(int d, int dm) { return fwd_table<kNormLinf>(d, dm); }

}  // namespace lip
