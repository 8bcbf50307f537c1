// Instances of the contraction kernel family: fp32, element-major layout.
#include "contract_dispatch.h"

namespace lpx {

ContractFn contract_kernel_fp32_em(int ntmax, int tile, int pf, int un) {
    return dispatch::by_nt<LPX_FP32, LPX_ELEMENT_MAJOR>(ntmax, tile, pf, un);
}

}  // namespace lpx
