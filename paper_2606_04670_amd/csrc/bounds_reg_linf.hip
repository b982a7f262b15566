// Instantiation unit of the regional-monotonicity bound kernel for one norm
// (all d and free-coordinate counts).
#include "bounds_reg.hpp"

namespace lip {

RegLaunch reg_linf(int d, int df) { return reg_table<kNormLinf>(d, df); }

}  // namespace lip
