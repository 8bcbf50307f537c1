// Instances of the contraction kernel family: fp32, DOF-major layout.
#include "contract_dispatch.h"

namespace lpx {

ContractFn contract_kernel_fp32_dm(int ntmax, int tile, int pf, int un) {
    return dispatch::by_nt<LPX_FP32, LPX_DOF_MAJOR>(ntmax, tile, pf, un);
}

}  // namespace lpx
