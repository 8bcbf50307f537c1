// Instances of the batch-run kernels (runs of consecutive tiles of the
// instances of a ragged batch): bf16, DOF-major layout, i-block bound LPX_NT
// (this unit is compiled once for each of 2, 4 and 8).
#include "contract_dispatch.h"

#ifndef LPX_NT
#error "compile with -DLPX_NT=2, 4 or 8"
#endif

namespace lpx {

template RunsFn runs_instances<LPX_BF16, LPX_DOF_MAJOR, LPX_NT>(int, int, int);

}  // namespace lpx
