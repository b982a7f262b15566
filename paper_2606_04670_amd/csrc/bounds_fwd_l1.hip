// Instantiation unit of the fused bound kernels (plain and batched) for one
// norm (all d, all monotone-coordinate counts).
#include "bounds_fwd.hpp"

namespace lip {

FwdLaunchers fwd_launchers_l1(int d, int dm) { return fwd_table<kNormL1>(d, dm); }

}  // namespace lip
