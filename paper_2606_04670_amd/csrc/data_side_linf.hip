// Instantiation unit of the FP64 data-side kernels for one norm (all d,
// with and without distance weights).
#include "data_side.hpp"

namespace lip {

bool ds_table_linf(int d, bool hasw, DsLaunchers *L) { return ds_table<3>(d, hasw, L); }

}  // namespace lip
