// Instantiation unit of the regional-monotonicity bound kernel for one norm
// (all d and free-coordinate counts).
#include "bounds_reg.hpp"

namespace lip {

RegLaunch reg_l1(int d, int df) { return reg_table<kNormL1>(d, df); }

}  // namespace lip
