// Instantiation unit of the smoothing-objective kernel for one norm (all d
// and monotone counts, global and per-datum constants, all pairs and
// pre-screened).
#include "smooth.hpp"

namespace lip {

SmoothLaunch smooth_linf(int d, int dm, bool local, bool prune)
{
    return smooth_table<3>(d, dm, local, prune);
}

}  // namespace lip
