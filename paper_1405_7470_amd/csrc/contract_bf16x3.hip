// Instantiations of the contraction kernel family for precision BF16X3.
#include "contract_kernels.h"

namespace lpx {

using ContractFn = void (*)(kern::ContractArgs);

namespace {
template <int LAYOUT, int NTMAX, int TILE_E, int PF, int UN>
ContractFn fn() {
    return &kern::contract_kernel<LPX_BF16X3, LAYOUT, NTMAX, TILE_E, PF, UN>;
}

template <int LAYOUT, int NTMAX, int TILE_E, int PF>
ContractFn by_unroll(int un) {
    switch (un) {
        case 1: return fn<LAYOUT, NTMAX, TILE_E, PF, 1>();
        case 2: return fn<LAYOUT, NTMAX, TILE_E, PF, 2>();
        default: return fn<LAYOUT, NTMAX, TILE_E, PF, 4>();
    }
}

template <int LAYOUT, int NTMAX, int TILE_E>
ContractFn by_prefetch(int pf, int un) {
    switch (pf) {
        case 0: return by_unroll<LAYOUT, NTMAX, TILE_E, 0>(un);
        case 1: return by_unroll<LAYOUT, NTMAX, TILE_E, 1>(un);
        case 2: return by_unroll<LAYOUT, NTMAX, TILE_E, 2>(un);
        case 3: return by_unroll<LAYOUT, NTMAX, TILE_E, 3>(un);
        default: break;
    }
    // D in registers: built only where the fragments fit (Np <= 64, four
    // waves per block); the unroll knob does not apply (fully unrolled).
    if constexpr (NTMAX <= 4) {
        if (pf == 4) return fn<LAYOUT, NTMAX, TILE_E, 4, 1>();
        if constexpr (contract_shape(TILE_E, NTMAX, 6).wpe == 4)
            if (pf == 6) return fn<LAYOUT, NTMAX, TILE_E, 6, 1>();
    }
    return nullptr;
}

template <int LAYOUT, int NTMAX>
ContractFn by_tile(int tile, int pf, int un) {
    switch (tile) {
        case 16: return by_prefetch<LAYOUT, NTMAX, 16>(pf, un);
        case 32: return by_prefetch<LAYOUT, NTMAX, 32>(pf, un);
        default: return by_prefetch<LAYOUT, NTMAX, 64>(pf, un);
    }
}

template <int LAYOUT>
ContractFn by_nt(int ntmax, int tile, int pf, int un) {
    switch (ntmax) {
        case 2: return by_tile<LAYOUT, 2>(tile, pf, un);
        case 4: return by_tile<LAYOUT, 4>(tile, pf, un);
        default: return by_tile<LAYOUT, 8>(tile, pf, un);
    }
}
}  // namespace

ContractFn contract_kernel_bf16x3(int layout, int ntmax, int tile, int pf, int un) {
    return layout == LPX_ELEMENT_MAJOR ? by_nt<LPX_ELEMENT_MAJOR>(ntmax, tile, pf, un)
                                       : by_nt<LPX_DOF_MAJOR>(ntmax, tile, pf, un);
}

}  // namespace lpx
