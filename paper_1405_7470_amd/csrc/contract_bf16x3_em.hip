// Instances of the contraction kernel family: bf16x3, element-major layout.
#include "contract_dispatch.h"

namespace lpx {

ContractFn contract_kernel_bf16x3_em(int ntmax, int tile, int pf, int un) {
    return dispatch::by_nt<LPX_BF16X3, LPX_ELEMENT_MAJOR>(ntmax, tile, pf, un);
}

}  // namespace lpx
