// Instances of the dG volume kernels (the contraction with the metric
// applied by the store waves): bf16x3, DOF-major layout, i-block bound LPX_NT
// (this unit is compiled once for each of 2, 4 and 8).
#include "contract_dispatch.h"

#ifndef LPX_NT
#error "compile with -DLPX_NT=2, 4 or 8"
#endif

namespace lpx {

template ContractFn dg_instances<LPX_BF16X3, LPX_DOF_MAJOR, LPX_NT>(int, int, int);

}  // namespace lpx
