// Instantiation unit of the step-function bound kernel for one norm (all d
// and monotone counts).
#include "local_fwd.hpp"

namespace lip {

StepLaunch step_fwd_l1(int d, int dm) { return step_fwd_table<1>(d, dm); }

}  // namespace lip
