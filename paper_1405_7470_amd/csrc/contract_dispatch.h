// Record -> kernel instance table of the contraction family.  Records
// outside what is built map to nullptr.
#pragma once

#include "contract_kernels.h"

namespace lpx {

using ContractFn = void (*)(kern::ContractArgs);
using RunsFn = void (*)(kern::RunArgs);

namespace dispatch {

// The two kernels built for every record: one contraction, and the runs of
// a ragged batch.
struct Single {
    using Fn = ContractFn;
    template <int PREC, int LAYOUT, int NTMAX, int TILE_E, int PF, int UN>
    static Fn get() {
        return &kern::contract_kernel<PREC, LAYOUT, NTMAX, TILE_E, PF, UN>;
    }
};
struct Runs {
    using Fn = RunsFn;
    template <int PREC, int LAYOUT, int NTMAX, int TILE_E, int PF, int UN>
    static Fn get() {
        return &kern::contract_runs_kernel<PREC, LAYOUT, NTMAX, TILE_E, PF, UN>;
    }
};

template <class M, int PREC, int LAYOUT, int NTMAX, int TILE_E, int PF>
typename M::Fn by_unroll(int un) {
    switch (un) {
        case 1: return M::template get<PREC, LAYOUT, NTMAX, TILE_E, PF, 1>();
        case 2: return M::template get<PREC, LAYOUT, NTMAX, TILE_E, PF, 2>();
        default: return M::template get<PREC, LAYOUT, NTMAX, TILE_E, PF, 4>();
    }
}

template <class M, int PREC, int LAYOUT, int NTMAX, int TILE_E>
typename M::Fn by_prefetch(int pf, int un) {
    switch (pf) {
        case 0: return by_unroll<M, PREC, LAYOUT, NTMAX, TILE_E, 0>(un);
        case 1: return by_unroll<M, PREC, LAYOUT, NTMAX, TILE_E, 1>(un);
        case 2: return by_unroll<M, PREC, LAYOUT, NTMAX, TILE_E, 2>(un);
        case 3: return by_unroll<M, PREC, LAYOUT, NTMAX, TILE_E, 3>(un);
        case 10: return by_unroll<M, PREC, LAYOUT, NTMAX, TILE_E, 10>(un);
        case 11: return by_unroll<M, PREC, LAYOUT, NTMAX, TILE_E, 11>(un);
        default: break;
    }
    // D in registers: built only where the fragments fit (Np <= 64); the
    // unroll knob does not apply (fully unrolled).
    if constexpr (NTMAX <= 4) {
        if (pf == 4) return M::template get<PREC, LAYOUT, NTMAX, TILE_E, 4, 1>();
        if (pf == 6) return M::template get<PREC, LAYOUT, NTMAX, TILE_E, 6, 1>();
        if (pf == 14) return M::template get<PREC, LAYOUT, NTMAX, TILE_E, 14, 1>();
    }
    return nullptr;
}

template <class M, int PREC, int LAYOUT, int NTMAX>
typename M::Fn by_tile(int tile, int pf, int un) {
    switch (tile) {
        case 16: return by_prefetch<M, PREC, LAYOUT, NTMAX, 16>(pf, un);
        case 32: return by_prefetch<M, PREC, LAYOUT, NTMAX, 32>(pf, un);
        default: return by_prefetch<M, PREC, LAYOUT, NTMAX, 64>(pf, un);
    }
}

// dG volume term (EPI = 1): only the staged-output records, prefetch 10, 11
// and 14, carry the epilogue.
template <int PREC, int LAYOUT, int NTMAX, int TILE_E, int PF>
ContractFn dg_by_unroll(int un) {
    switch (un) {
        case 1: return &kern::contract_kernel<PREC, LAYOUT, NTMAX, TILE_E, PF, 1, 1>;
        case 2: return &kern::contract_kernel<PREC, LAYOUT, NTMAX, TILE_E, PF, 2, 1>;
        default: return &kern::contract_kernel<PREC, LAYOUT, NTMAX, TILE_E, PF, 4, 1>;
    }
}

template <int PREC, int LAYOUT, int NTMAX, int TILE_E>
ContractFn dg_by_prefetch(int pf, int un) {
    if (pf == 10) return dg_by_unroll<PREC, LAYOUT, NTMAX, TILE_E, 10>(un);
    if (pf == 11) return dg_by_unroll<PREC, LAYOUT, NTMAX, TILE_E, 11>(un);
    if constexpr (NTMAX <= 4) {
        if (pf == 14) return &kern::contract_kernel<PREC, LAYOUT, NTMAX, TILE_E, 14, 1, 1>;
    }
    return nullptr;
}

template <int PREC, int LAYOUT, int NTMAX>
ContractFn dg_by_tile(int tile, int pf, int un) {
    switch (tile) {
        case 16: return dg_by_prefetch<PREC, LAYOUT, NTMAX, 16>(pf, un);
        case 32: return dg_by_prefetch<PREC, LAYOUT, NTMAX, 32>(pf, un);
        default: return dg_by_prefetch<PREC, LAYOUT, NTMAX, 64>(pf, un);
    }
}

}  // namespace dispatch

// The instances of one (precision, layout, i-block bound NTMAX): each
// instance unit (contract_<precision>_<layout>.hip) is compiled once per
// bound, 2, 4 and 8, with -DLPX_NT, so that the instances compile in
// parallel; everywhere else these are extern.
template <int PREC, int LAYOUT, int NTMAX>
ContractFn contract_instances(int tile, int pf, int un) {
    return dispatch::by_tile<dispatch::Single, PREC, LAYOUT, NTMAX>(tile, pf, un);
}

// The batch-run instances, compiled the same way by the units
// contract_runs_<precision>_<layout>.hip.
template <int PREC, int LAYOUT, int NTMAX>
RunsFn runs_instances(int tile, int pf, int un) {
    return dispatch::by_tile<dispatch::Runs, PREC, LAYOUT, NTMAX>(tile, pf, un);
}

// The dG volume instances, compiled the same way by the units
// contract_dg_<precision>_<layout>.hip.
template <int PREC, int LAYOUT, int NTMAX>
ContractFn dg_instances(int tile, int pf, int un) {
    return dispatch::dg_by_tile<PREC, LAYOUT, NTMAX>(tile, pf, un);
}

#define LPX_EXTERN_INSTANCES(P, L)                                               \
    extern template ContractFn contract_instances<P, L, 2>(int, int, int);    \
    extern template ContractFn contract_instances<P, L, 4>(int, int, int);    \
    extern template ContractFn contract_instances<P, L, 8>(int, int, int);    \
    extern template ContractFn dg_instances<P, L, 2>(int, int, int);          \
    extern template ContractFn dg_instances<P, L, 4>(int, int, int);          \
    extern template ContractFn dg_instances<P, L, 8>(int, int, int);          \
    extern template RunsFn runs_instances<P, L, 2>(int, int, int);            \
    extern template RunsFn runs_instances<P, L, 4>(int, int, int);            \
    extern template RunsFn runs_instances<P, L, 8>(int, int, int);
LPX_EXTERN_INSTANCES(LPX_FP32, LPX_ELEMENT_MAJOR)
LPX_EXTERN_INSTANCES(LPX_FP32, LPX_DOF_MAJOR)
LPX_EXTERN_INSTANCES(LPX_BF16, LPX_ELEMENT_MAJOR)
LPX_EXTERN_INSTANCES(LPX_BF16, LPX_DOF_MAJOR)
LPX_EXTERN_INSTANCES(LPX_BF16X3, LPX_ELEMENT_MAJOR)
LPX_EXTERN_INSTANCES(LPX_BF16X3, LPX_DOF_MAJOR)
#undef LPX_EXTERN_INSTANCES

// Record -> instance for a run-time bound (dg: the dG volume epilogue).
template <int PREC, int LAYOUT>
ContractFn contract_instance(int ntmax, int tile, int pf, int un, bool dg = false) {
    if (dg) {
        switch (ntmax) {
            case 2: return dg_instances<PREC, LAYOUT, 2>(tile, pf, un);
            case 4: return dg_instances<PREC, LAYOUT, 4>(tile, pf, un);
            default: return dg_instances<PREC, LAYOUT, 8>(tile, pf, un);
        }
    }
    switch (ntmax) {
        case 2: return contract_instances<PREC, LAYOUT, 2>(tile, pf, un);
        case 4: return contract_instances<PREC, LAYOUT, 4>(tile, pf, un);
        default: return contract_instances<PREC, LAYOUT, 8>(tile, pf, un);
    }
}

// Batch-run instance of a record for a run-time bound.
template <int PREC, int LAYOUT>
RunsFn runs_instance(int ntmax, int tile, int pf, int un) {
    switch (ntmax) {
        case 2: return runs_instances<PREC, LAYOUT, 2>(tile, pf, un);
        case 4: return runs_instances<PREC, LAYOUT, 4>(tile, pf, un);
        default: return runs_instances<PREC, LAYOUT, 8>(tile, pf, un);
    }
}

// Kernel arguments of one validated contraction (Darr and G left NULL).
kern::ContractArgs contract_args(const lpx_contract_desc& c, const ContractGeom& g);

// Resident work-groups per CU of kernel `fn` with `threads` threads and
// `lds` bytes of dynamic LDS on `device` (cached; sets the kernel's LDS
// limit attribute when above 64 KiB).
lpx_status blocks_per_cu(const void* fn, int threads, int64_t lds, int device, int* out);

}  // namespace lpx
