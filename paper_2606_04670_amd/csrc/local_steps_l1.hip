// Instantiation unit of the step-function kernels (table builder and bounds)
// for one norm (all d, with and without distance weights, 4 or 8 knot slots).
#include "local_steps.hpp"

namespace lip {

bool step_table_l1(int d, bool hasw, int kb, StepLaunchers *L) { return step_table<1>(d, hasw, kb, L); }

}  // namespace lip
