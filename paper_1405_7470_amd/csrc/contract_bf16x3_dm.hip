// Instances of the contraction kernel family: bf16x3, DOF-major layout.
#include "contract_dispatch.h"

namespace lpx {

ContractFn contract_kernel_bf16x3_dm(int ntmax, int tile, int pf, int un) {
    return dispatch::by_nt<LPX_BF16X3, LPX_DOF_MAJOR>(ntmax, tile, pf, un);
}

}  // namespace lpx
