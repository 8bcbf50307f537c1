// Surface term of a nodal dG operator (Table 1's "dG FEM surface"): each
// element's face fluxes, scaled by a per-face factor, lifted into the
// element by one rectangular operator L [Np][M], M = nf * nfp:
//
//     out[e,i] = sum_{m<M} L[i][m] * fl32(s(e, m / nfp) * f(e, m))
//
// The contraction with a non-square operator and a fused input scaling.
// MFMA layout as in the contraction kernels (contract_kernels.h): 16-row
// blocks of L (nrb = ceil(Np/16)) against 16-element blocks, FP32 k-steps
// of 4 columns (column 4s + g for lane group g) or bf16 k-steps of 32
// (columns 32s + 8g .. +7).  L is staged once per work-group in LDS in MFMA
// operand order, converted to the operand precision (the record's prefetch
// bit 0, the only staging built).  Each wave takes tile_e / 16 element blocks
// at a time (the record's tile_e), so every L fragment read from LDS feeds
// that many MFMAs; the flux operand is read from global memory, scaled in
// FP32 and converted in registers.  Every record of a precision sums each
// output in column order with the same operations, so records of one
// precision agree bit for bit.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "contract_kernels.h"

namespace lpx {
namespace liftk {

using kern::f4;
using kern::Frag;
constexpr int kThreads = 256, kWaves = 4;

struct Args {
    const float* __restrict__ L;
    const float* __restrict__ f;
    const float* __restrict__ sc;
    float* __restrict__ out;
    int64_t E, nblocks;
    int Np, nf, nfp, M, nrb, nsteps;
    Divider nfp_div;  // m -> face m / nfp
    int np_vec, e_vec;
};

__device__ __forceinline__ int face_of(const Args& a, int m) {
    return (int)(((uint64_t)(uint32_t)m * a.nfp_div.m) >> a.nfp_div.sh);
}

// Scaled flux fl32(s(e, m / nfp) * f(e, m)) for one lane; zero past the
// element range or column range (reads are clamped in bounds, never branched).
template <int LAYOUT>
__device__ __forceinline__ float scaled(const Args& a, int64_t e, int m) {
    const bool ok = e < a.E && m < a.M;
    const int64_t ec = e < a.E ? e : a.E - 1;
    const int mc = m < a.M ? m : a.M - 1;
    const int c = face_of(a, mc);
    const float fv = LAYOUT == LPX_ELEMENT_MAJOR ? a.f[ec * a.M + mc] : a.f[(int64_t)mc * a.E + ec];
    const float sv = LAYOUT == LPX_ELEMENT_MAJOR ? a.sc[ec * a.nf + c] : a.sc[(int64_t)c * a.E + ec];
    const float g = sv * fv;
    return ok ? g : 0.0f;
}

// L fragment (row block p, step s, lane l) from global memory.
template <int PREC>
__device__ __forceinline__ Frag<PREC> l_frag_global(const Args& a, int p, int s, int l) {
    const int i = 16 * p + (l & 15);
    const int ic = i < a.Np ? i : a.Np - 1;
    if constexpr (PREC == LPX_FP32) {
        const int m = 4 * s + (l >> 4);
        const float x = a.L[(int64_t)ic * a.M + (m < a.M ? m : a.M - 1)];
        return {i < a.Np && m < a.M ? x : 0.0f};
    } else {
        float v[8];
        const int m0 = 32 * s + 8 * (l >> 4);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int m = m0 + t;
            const float x = a.L[(int64_t)ic * a.M + (m < a.M ? m : a.M - 1)];
            v[t] = i < a.Np && m < a.M ? x : 0.0f;
        }
        return kern::make_frag8<PREC>(v);
    }
}

// Flux operand of the block starting at e0, step s.
template <int PREC, int LAYOUT>
__device__ __forceinline__ Frag<PREC> f_frag(const Args& a, int64_t e0, int s, int l) {
    const int64_t e = e0 + (l & 15);
    if constexpr (PREC == LPX_FP32) {
        return {scaled<LAYOUT>(a, e, 4 * s + (l >> 4))};
    } else {
        float v[8];
        const int m0 = 32 * s + 8 * (l >> 4);
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = scaled<LAYOUT>(a, e, m0 + t);
        return kern::make_frag8<PREC>(v);
    }
}

template <int PREC, int LAYOUT, int NT, int BPW>
__global__ __launch_bounds__(kThreads) void lift_kernel(Args a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t nfrag = (int64_t)a.nrb * a.nsteps * 64;
    // stage L in MFMA operand order (the contraction's D layout)
    for (int64_t idx = tid; idx < nfrag; idx += kThreads) {
        const int l = (int)(idx & 63), rest = (int)(idx >> 6);
        const int s = rest % a.nsteps, p = rest / a.nsteps;
        kern::d_frag_store_lds<PREC>(lds, nfrag, (int)idx, l_frag_global<PREC>(a, p, s, l));
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kWaves * BPW;
    for (int64_t b0 = ((int64_t)blockIdx.x * kWaves + wave) * BPW; b0 < a.nblocks; b0 += stride) {
        f4 acc[BPW][NT];
#pragma unroll
        for (int b = 0; b < BPW; ++b)
#pragma unroll
            for (int p = 0; p < NT; ++p) acc[b][p] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int s = 0; s < a.nsteps; ++s) {
            Frag<PREC> uf[BPW];
#pragma unroll
            for (int b = 0; b < BPW; ++b) uf[b] = f_frag<PREC, LAYOUT>(a, 16 * (b0 + b), s, lane);
#pragma unroll
            for (int p = 0; p < NT; ++p) {
                // row blocks past nrb hold a clamped duplicate, never stored
                const int pc = p < a.nrb ? p : a.nrb - 1;
                const Frag<PREC> df = kern::d_frag_lds<PREC>(lds, nfrag, (pc * a.nsteps + s) * 64 + lane);
#pragma unroll
                for (int b = 0; b < BPW; ++b) {
                    if constexpr (LAYOUT == LPX_ELEMENT_MAJOR)
                        acc[b][p] = kern::mma(df, uf[b], acc[b][p]);  // rows i, columns e
                    else
                        acc[b][p] = kern::mma(uf[b], df, acc[b][p]);  // rows e, columns i
                }
            }
        }
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
            const int64_t eb = 16 * (b0 + b);
            if (b0 + b >= a.nblocks) continue;
#pragma unroll
            for (int p = 0; p < NT; ++p) {
                if (p >= a.nrb) continue;
                if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
                    const int64_t e = eb + (lane & 15);
                    const int i0 = 16 * p + 4 * (lane >> 4);
                    if (e >= a.E) continue;
                    float* dst = a.out + e * a.Np + i0;
                    if (a.np_vec) {
                        if (i0 < a.Np) *reinterpret_cast<f4*>(dst) = acc[b][p];
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (i0 + r < a.Np) dst[r] = acc[b][p][r];
                    }
                } else {
                    const int i = 16 * p + (lane & 15);
                    const int64_t e = eb + 4 * (lane >> 4);
                    if (i >= a.Np || e >= a.E) continue;
                    float* dst = a.out + (int64_t)i * a.E + e;
                    if (a.e_vec) {
                        *reinterpret_cast<f4*>(dst) = acc[b][p];
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (e + r < a.E) dst[r] = acc[b][p][r];
                    }
                }
            }
        }
    }
}

using Fn = void (*)(Args);

template <int PREC, int LAYOUT, int NT>
Fn by_bpw(int bpw) {
    switch (bpw) {
        case 1: return &lift_kernel<PREC, LAYOUT, NT, 1>;
        case 2: return &lift_kernel<PREC, LAYOUT, NT, 2>;
        default: return &lift_kernel<PREC, LAYOUT, NT, 4>;
    }
}

template <int PREC, int LAYOUT>
Fn by_nt(int nt, int bpw) {
    switch (nt) {
        case 2: return by_bpw<PREC, LAYOUT, 2>(bpw);
        case 4: return by_bpw<PREC, LAYOUT, 4>(bpw);
        default: return by_bpw<PREC, LAYOUT, 8>(bpw);
    }
}

Fn select(int prec, int layout, int nt, int bpw) {
    const bool em = layout == LPX_ELEMENT_MAJOR;
    switch (prec) {
        case LPX_FP32:
            return em ? by_nt<LPX_FP32, LPX_ELEMENT_MAJOR>(nt, bpw)
                      : by_nt<LPX_FP32, LPX_DOF_MAJOR>(nt, bpw);
        case LPX_BF16:
            return em ? by_nt<LPX_BF16, LPX_ELEMENT_MAJOR>(nt, bpw)
                      : by_nt<LPX_BF16, LPX_DOF_MAJOR>(nt, bpw);
        default:
            return em ? by_nt<LPX_BF16X3, LPX_ELEMENT_MAJOR>(nt, bpw)
                      : by_nt<LPX_BF16X3, LPX_DOF_MAJOR>(nt, bpw);
    }
}

struct Geom {
    lpx_record r;
    int nt, nrb, nsteps;
    int64_t lds, nblocks;
};

}  // namespace liftk

static lpx_status validate_lift(const lpx_dg_surface_desc* c, const lpx_record* rec,
                                liftk::Geom* g, bool* noop) {
    *noop = true;
    if (!c) return set_error(LPX_ERR_INVALID_ARG, "descriptor is NULL");
    lpx_record r = rec ? *rec : default_record(LPX_FP32);
    if (!rec) r.prefetch = 1;
    lpx_status s = check_record(&r);
    if (s != LPX_OK) return s;
    if (r.prefetch != 1)
        return set_error(LPX_ERR_UNSUPPORTED,
                         "the lift stages its operator in LDS: prefetch must be 1, got %u",
                         r.prefetch);
    if (c->Np < 0 || c->nf < 0 || c->nfp < 0 || c->E < 0)
        return set_error(LPX_ERR_INVALID_ARG, "negative size");
    if (c->layout != LPX_ELEMENT_MAJOR && c->layout != LPX_DOF_MAJOR)
        return set_error(LPX_ERR_INVALID_ARG, "unknown layout %d", c->layout);
    if (c->reserved != 0) return set_error(LPX_ERR_INVALID_ARG, "reserved must be 0");
    if (c->Np > kMaxNp) return set_error(LPX_ERR_UNSUPPORTED, "Np=%d above %d", c->Np, kMaxNp);
    const int64_t M = (int64_t)c->nf * c->nfp;
    if (M > 4096) return set_error(LPX_ERR_UNSUPPORTED, "nf*nfp = %lld above 4096", (long long)M);
    int64_t felems, oelems;
    if (mul_overflows(c->E, M, &felems) || mul_overflows(c->E, c->Np, &oelems) ||
        felems > INT64_MAX / 4 || oelems > INT64_MAX / 4)
        return set_error(LPX_ERR_INVALID_ARG, "size product overflows int64");
    g->r = r;
    g->nrb = (int)ceil_div(c->Np, 16);
    g->nt = g->nrb <= 2 ? 2 : (g->nrb <= 4 ? 4 : 8);
    g->nsteps = (int)ceil_div(M, r.precision == LPX_FP32 ? 4 : 32);
    const int64_t frag_bytes = r.precision == LPX_FP32 ? 4 : (r.precision == LPX_BF16 ? 16 : 32);
    g->lds = (int64_t)g->nrb * g->nsteps * 64 * frag_bytes;
    g->nblocks = ceil_div(c->E, 16);
    if (g->lds > kMaxLdsPerWorkgroup)
        return set_error(LPX_ERR_UNSUPPORTED,
                         "the lift's operator needs %lld bytes of LDS (limit %lld)",
                         (long long)g->lds, (long long)kMaxLdsPerWorkgroup);
    if (c->Np == 0 || M == 0 || c->E == 0) return LPX_OK;
    if (!c->L || !c->f || !c->s || !c->out)
        return set_error(LPX_ERR_INVALID_ARG, "NULL L, f, s or out");
    const void* ptrs[] = {c->L, c->f, c->s, c->out};
    for (const void* p : ptrs)
        if (reinterpret_cast<uintptr_t>(p) & 15u)
            return set_error(LPX_ERR_INVALID_ARG, "L, f, s and out must be 16-byte aligned");
    const int64_t ob = oelems * 4;
    if (overlaps(c->out, ob, c->L, (int64_t)c->Np * M * 4) || overlaps(c->out, ob, c->f, felems * 4) ||
        overlaps(c->out, ob, c->s, c->E * c->nf * 4))
        return set_error(LPX_ERR_ALIAS, "out overlaps L, f or s");
    *noop = false;
    return LPX_OK;
}

}  // namespace lpx

using namespace lpx;

extern "C" {

lpx_status lpx_dg_surface_validate(const lpx_dg_surface_desc* c, const lpx_record* rec) {
    clear_error();
    try {
        liftk::Geom g;
        bool noop;
        return validate_lift(c, rec, &g, &noop);
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_dg_surface(const lpx_dg_surface_desc* c, const lpx_record* rec, void* stream) {
    clear_error();
    try {
        liftk::Geom g;
        bool noop;
        lpx_status s = validate_lift(c, rec, &g, &noop);
        if (s != LPX_OK || noop) return s;
        DeviceInfo dev;
        if ((s = current_device_info(&dev)) != LPX_OK) return s;
        const int bpw = g.r.tile_e / 16;
        liftk::Fn fn = liftk::select(g.r.precision, c->layout, g.nt, bpw);
        const void* fp = reinterpret_cast<const void*>(fn);
        static std::mutex mu;
        static std::map<std::pair<const void*, int>, int> occ;  // (kernel, device) -> blocks/CU
        int nb = 0;
        {
            std::lock_guard<std::mutex> lock(mu);
            auto key = std::make_pair(fp, dev.device);
            auto it = occ.find(key);
            if (it != occ.end()) {
                nb = it->second;
            } else {
                hipError_t e = hipFuncSetAttribute(fp, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)kMaxLdsPerWorkgroup);
                if (e == hipSuccess)
                    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fp, liftk::kThreads,
                                                                     (size_t)g.lds);
                if (e != hipSuccess)
                    return set_error(LPX_ERR_HIP, "lift occupancy: %s", hipGetErrorString(e));
                occ[key] = nb;
            }
        }
        if (nb <= 0) return set_error(LPX_ERR_UNSUPPORTED, "lift kernel cannot be resident");
        int64_t grid = (int64_t)nb * dev.num_cu;
        const int64_t need = ceil_div(g.nblocks, (int64_t)liftk::kWaves * bpw);
        if (grid > need) grid = need;
        liftk::Args a;
        a.L = c->L;
        a.f = c->f;
        a.sc = c->s;
        a.out = c->out;
        a.E = c->E;
        a.nblocks = g.nblocks;
        a.Np = c->Np;
        a.nf = c->nf;
        a.nfp = c->nfp;
        a.M = c->nf * c->nfp;
        a.nrb = g.nrb;
        a.nsteps = g.nsteps;
        a.nfp_div = make_divider(c->nfp);
        a.np_vec = c->Np % 4 == 0;
        a.e_vec = c->E % 4 == 0;
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(liftk::kThreads), (size_t)g.lds,
                           reinterpret_cast<hipStream_t>(stream), a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return set_error(LPX_ERR_HIP, "lift launch: %s", hipGetErrorString(e));
        return LPX_OK;
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

}  // extern "C"
