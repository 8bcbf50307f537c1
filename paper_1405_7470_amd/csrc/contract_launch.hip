// Launch of the contraction kernel family: record -> kernel instance, grid.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "contract_dispatch.h"

namespace lpx {

namespace {

ContractFn select(const ContractGeom& g) {
    const bool em = g.layout == LPX_ELEMENT_MAJOR, dg = g.dg != 0;
    const int nt = g.ntmax, t = g.tile_e, pf = g.prefetch, un = g.unroll;
    switch (g.prec) {
        case LPX_FP32:
            return em ? contract_instance<LPX_FP32, LPX_ELEMENT_MAJOR>(nt, t, pf, un, dg)
                      : contract_instance<LPX_FP32, LPX_DOF_MAJOR>(nt, t, pf, un, dg);
        case LPX_BF16:
            return em ? contract_instance<LPX_BF16, LPX_ELEMENT_MAJOR>(nt, t, pf, un, dg)
                      : contract_instance<LPX_BF16, LPX_DOF_MAJOR>(nt, t, pf, un, dg);
        default:
            return em ? contract_instance<LPX_BF16X3, LPX_ELEMENT_MAJOR>(nt, t, pf, un, dg)
                      : contract_instance<LPX_BF16X3, LPX_DOF_MAJOR>(nt, t, pf, un, dg);
    }
}

}  // namespace

lpx_status blocks_per_cu(const void* fn, int threads, int64_t lds, int device, int* out) {
    static std::mutex mu;
    static std::map<std::pair<std::pair<const void*, int64_t>, int>, int> cache;
    static std::map<std::pair<const void*, int>, bool> lds_attr_set;
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(std::make_pair(fn, lds), device);
    auto it = cache.find(key);
    if (it != cache.end()) {
        *out = it->second;
        return LPX_OK;
    }
    if (lds > 64 * 1024 && !lds_attr_set[{fn, device}]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)kMaxLdsPerWorkgroup);
        if (e != hipSuccess)
            return set_error(LPX_ERR_HIP, "hipFuncSetAttribute: %s", hipGetErrorString(e));
        lds_attr_set[{fn, device}] = true;
    }
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, (size_t)lds);
    if (e != hipSuccess)
        return set_error(LPX_ERR_HIP, "hipOccupancyMaxActiveBlocksPerMultiprocessor: %s",
                         hipGetErrorString(e));
    cache[key] = nb;
    *out = nb;
    return LPX_OK;
}

namespace {

// Device scratch for lpx_contract_noalloc: D's MFMA-order arrangement of
// records that read D from memory goes here instead of into a workspace
// allocated per call.  Every GPU the library runs on holds one copy until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// the device address: the address is looked up once per device with
// hipGetSymbolAddress and only that pointer is passed to kernels.
__device__ __align__(256) unsigned char scratch[LPX_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch;  // device -> address of its `scratch`

lpx_status scratch_address(unsigned char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(LPX_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return LPX_OK;
    }
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        return set_error(LPX_ERR_HIP, "hipGetSymbolAddress(scratch): %s",
                         e != hipSuccess ? hipGetErrorString(e) : "null address");
    g_scratch[dev] = static_cast<unsigned char*>(p);
    *out = g_scratch[dev];
    return LPX_OK;
}

}  // namespace

int64_t darr_bytes(const ContractGeom& g) {
    if (g.prefetch & 5) return 0;  // D in LDS or registers: no arrangement in memory
    const int64_t frag_bytes = g.prec == LPX_FP32 ? 4 : (g.prec == LPX_BF16 ? 16 : 32);
    return g.nfrag * frag_bytes;
}

kern::ContractArgs contract_args(const lpx_contract_desc& c, const ContractGeom& g) {
    kern::ContractArgs a;
    a.D = c.D;
    a.Darr = nullptr;
    a.u = c.u;
    a.out = c.out;
    a.E = c.E;
    a.ntiles = g.ntiles;
    a.K = c.K;
    a.Np = c.Np;
    a.nt = g.nt;
    a.nrb = g.nrb;
    a.np_div = make_divider(c.Np);
    a.nsteps = g.nsteps;
    a.ldu = g.ldu;
    a.ldo = g.ldo;
    a.G = nullptr;
    a.ldo_g = g.ldo_g;
    a.np_vec = (c.Np % 4) == 0;
    a.e_vec = (c.E % 4) == 0;
    a.stream_out = (int64_t)c.K * c.E * c.Np * 4 >= ((int64_t)32 << 20);
    a.blocked = g.order;
    return a;
}

lpx_status launch_contract(const lpx_contract_desc& c, const ContractGeom& g, void* stream,
                           bool noalloc, const float* G) {
    DeviceInfo dev;
    lpx_status s = current_device_info(&dev);
    if (s != LPX_OK) return s;
    if (g.lds_bytes > dev.max_lds_per_block)
        return set_error(LPX_ERR_UNSUPPORTED, "needs %lld bytes of LDS, device allows %d",
                         (long long)g.lds_bytes, dev.max_lds_per_block);
    ContractFn fn = select(g);
    if (!fn) return set_error(LPX_ERR_INTERNAL, "no kernel instance for a validated record");
    int nb = 0;
    s = blocks_per_cu(reinterpret_cast<const void*>(fn), g.threads, g.lds_bytes, dev.device, &nb);
    if (s != LPX_OK) return s;
    if (nb <= 0)
        return set_error(LPX_ERR_UNSUPPORTED, "kernel cannot be resident (LDS %lld bytes)",
                         (long long)g.lds_bytes);
    int64_t grid = (int64_t)nb * dev.num_cu;
    if (grid > g.ntiles) grid = g.ntiles;

    kern::ContractArgs a = contract_args(c, g);
    a.G = G;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // Kernels that read D from memory read its MFMA-order arrangement,
    // written by a pre-pass into a stream-ordered workspace.
    unsigned char* darr = nullptr;
    const bool arrange = (g.prefetch & 5) == 0;
    const bool own_ws = arrange && !noalloc;  // a workspace this call allocates and frees
    if (arrange) {
        if (noalloc) {
            if (darr_bytes(g) > LPX_NOALLOC_SCRATCH_BYTES)
                return set_error(LPX_ERR_UNSUPPORTED, "D arrangement needs %lld bytes, scratch holds %d",
                                 (long long)darr_bytes(g), LPX_NOALLOC_SCRATCH_BYTES);
            s = scratch_address(&darr);
        } else {
            s = workspace_alloc((void**)&darr, (size_t)darr_bytes(g), stream, "D arrangement");
        }
        if (s != LPX_OK) return s;
        a.Darr = darr;
        const dim3 ag(kern::kArrangeBlocks), ab(kern::kArrangeThreads);
        if (g.prec == LPX_FP32)
            hipLaunchKernelGGL(kern::arrange_d_kernel<LPX_FP32>, ag, ab, 0, st, a, darr);
        else if (g.prec == LPX_BF16)
            hipLaunchKernelGGL(kern::arrange_d_kernel<LPX_BF16>, ag, ab, 0, st, a, darr);
        else
            hipLaunchKernelGGL(kern::arrange_d_kernel<LPX_BF16X3>, ag, ab, 0, st, a, darr);
    }
    void* args[] = {&a};
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)grid),
                            dim3(g.threads), args, (size_t)g.lds_bytes, st);
    if (e == hipSuccess) e = hipGetLastError();
    if (own_ws) {
        const hipError_t ef = hipFreeAsync(darr, st);
        if (e == hipSuccess) e = ef;
    }
    if (e != hipSuccess)
        return set_error(LPX_ERR_HIP, "contraction launch: %s", hipGetErrorString(e));
    return LPX_OK;
}

}  // namespace lpx
