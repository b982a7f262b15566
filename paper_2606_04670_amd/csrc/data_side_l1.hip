// Instantiation unit of the FP64 data-side kernels for one norm (all d,
// with and without distance weights).
#include "data_side.hpp"

namespace lip {

bool ds_table_l1(int d, bool hasw, DsLaunchers *L) { return ds_table<1>(d, hasw, L); }

}  // namespace lip
