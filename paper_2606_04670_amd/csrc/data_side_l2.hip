// Instantiation unit of the FP64 data-side kernels for one norm (all d,
// with and without distance weights).
#include "data_side.hpp"

namespace lip {

bool ds_table_l2(int d, bool hasw, DsLaunchers *L) { return ds_table<2>(d, hasw, L); }

}  // namespace lip
