// Instances of the contraction kernel family: bf16, element-major layout.
#include "contract_dispatch.h"

namespace lpx {

ContractFn contract_kernel_bf16_em(int ntmax, int tile, int pf, int un) {
    return dispatch::by_nt<LPX_BF16, LPX_ELEMENT_MAJOR>(ntmax, tile, pf, un);
}

}  // namespace lpx
