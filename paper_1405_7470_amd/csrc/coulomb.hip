// 3D Coulomb potential phi[t] = sum_{s, r_ts > 0} q_s / |x_t - y_s| on gfx950
// (Table 1's "3D Coulomb pot." workload, counted in pairs per second).
//
// The transformation record carries the variant, as for the contraction:
//   tile_e   : sources per tile = 16 * tile_e (256, 512, 1024): split_iname
//              of the source loop (sec. 2.4.1), the outer part walked by every
//              work-group in order;
//   prefetch : 2 (bit 1) stages each source tile in LDS (add_prefetch, sec.
//              2.4.4); 0 reads the sources straight from global memory, one
//              address for the whole wave (a broadcast through the caches);
//   unroll   : targets per thread, 1, 2 or 4 (the `ilp` tag, sec. 2.4.2):
//              one source read feeds that many independent pair updates;
//   layout   : LPX_ELEMENT_MAJOR = array of structures (16-byte records),
//              LPX_DOF_MAJOR = structure of arrays (sec. 2.4.3);
//   precision: FP32 only.
// Every record sums each target's pairs in increasing source order with the
// same FP32 operations, so all records give bit-identical results.
//
// Pair: d = y_s - x_t (3 subtractions), r2 = |d|^2 (one multiply, two fused
// multiply-adds), rinv = v_rsq_f32(r2), a select that drops r2 == 0, and
// phi += q * rinv (fused multiply-add).  The kernel is bound by the vector
// ALU (the reciprocal square root issues at a quarter of the FP32 rate).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lpx_internal.h"

namespace lpx {
namespace coul {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kThreads = 256;

struct Args {
    const float* __restrict__ tg;
    const float* __restrict__ sr;
    float* __restrict__ phi;
    int64_t nt, ns;
};

template <int LAYOUT>
__device__ __forceinline__ f4 source(const Args& a, int64_t s) {
    if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
        return reinterpret_cast<const f4*>(a.sr)[s];
    } else {
        return f4{a.sr[s], a.sr[a.ns + s], a.sr[2 * a.ns + s], a.sr[3 * a.ns + s]};
    }
}

// One pair update of ILP targets from source sv.
template <int ILP>
__device__ __forceinline__ void pairs(const f4& sv, const float (&x)[ILP], const float (&y)[ILP],
                                      const float (&z)[ILP], float (&acc)[ILP]) {
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
        const float dx = sv[0] - x[k], dy = sv[1] - y[k], dz = sv[2] - z[k];
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float ri = __builtin_amdgcn_rsqf(r2);
        acc[k] = fmaf(sv[3], r2 > 0.0f ? ri : 0.0f, acc[k]);
    }
}

template <int LAYOUT, int TILE_S, int ILP, bool STAGE>
__global__ __launch_bounds__(kThreads) void coulomb_kernel(Args a) {
    __shared__ f4 tile[STAGE ? TILE_S : 1];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kThreads * ILP + tid;
    float x[ILP], y[ILP], z[ILP], acc[ILP];
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
        int64_t t = base + (int64_t)kThreads * k;
        t = t < a.nt ? t : a.nt - 1;  // clamped: computed, never stored
        if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
            const f4 p = reinterpret_cast<const f4*>(a.tg)[t];
            x[k] = p[0], y[k] = p[1], z[k] = p[2];
        } else {
            x[k] = a.tg[t], y[k] = a.tg[a.nt + t], z[k] = a.tg[2 * a.nt + t];
        }
        acc[k] = 0.0f;
    }
    for (int64_t s0 = 0; s0 < a.ns; s0 += TILE_S) {
        const int n = a.ns - s0 < TILE_S ? (int)(a.ns - s0) : TILE_S;
        if constexpr (STAGE) {
            __syncthreads();  // the previous tile is no longer read
#pragma unroll
            for (int j = 0; j < TILE_S / kThreads; ++j) {
                const int i = tid + kThreads * j;
                tile[i] = source<LAYOUT>(a, s0 + (i < n ? i : n - 1));
            }
            __syncthreads();
        }
        auto src = [&](int j) {
            if constexpr (STAGE)
                return tile[j];
            else
                return source<LAYOUT>(a, s0 + j);
        };
        if (n == TILE_S) {  // uniform: whole tile, compile-time trip count
#pragma unroll 8
            for (int j = 0; j < TILE_S; ++j) pairs<ILP>(src(j), x, y, z, acc);
        } else {
            for (int j = 0; j < n; ++j) pairs<ILP>(src(j), x, y, z, acc);
        }
    }
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
        const int64_t t = base + (int64_t)kThreads * k;
        if (t < a.nt) a.phi[t] = acc[k];
    }
}

using Fn = void (*)(Args);

template <int LAYOUT, int TILE_S, bool STAGE>
Fn by_ilp(int ilp) {
    switch (ilp) {
        case 1: return &coulomb_kernel<LAYOUT, TILE_S, 1, STAGE>;
        case 2: return &coulomb_kernel<LAYOUT, TILE_S, 2, STAGE>;
        default: return &coulomb_kernel<LAYOUT, TILE_S, 4, STAGE>;
    }
}

template <int LAYOUT>
Fn by_tile(int tile_s, bool stage, int ilp) {
    switch (tile_s) {
        case 256: return stage ? by_ilp<LAYOUT, 256, true>(ilp) : by_ilp<LAYOUT, 256, false>(ilp);
        case 512: return stage ? by_ilp<LAYOUT, 512, true>(ilp) : by_ilp<LAYOUT, 512, false>(ilp);
        default: return stage ? by_ilp<LAYOUT, 1024, true>(ilp) : by_ilp<LAYOUT, 1024, false>(ilp);
    }
}

}  // namespace coul

// Every check of lpx_coulomb that needs no HIP call; *noop marks zero sizes.
static lpx_status validate_coulomb(const lpx_coulomb_desc* c, const lpx_record* rec, bool* noop) {
    *noop = true;
    if (!c) return set_error(LPX_ERR_INVALID_ARG, "descriptor is NULL");
    lpx_record r = rec ? *rec : default_record(LPX_FP32);
    lpx_status s = check_record(&r);
    if (s != LPX_OK) return s;
    if (r.precision != LPX_FP32)
        return set_error(LPX_ERR_UNSUPPORTED, "the Coulomb potential is built in FP32 only");
    if (r.prefetch != 0 && r.prefetch != 2)
        return set_error(LPX_ERR_UNSUPPORTED,
                         "Coulomb records stage the sources (prefetch 2) or not (0), got %u",
                         r.prefetch);
    if (c->nt < 0 || c->ns < 0) return set_error(LPX_ERR_INVALID_ARG, "negative size");
    if (c->layout != LPX_ELEMENT_MAJOR && c->layout != LPX_DOF_MAJOR)
        return set_error(LPX_ERR_INVALID_ARG, "unknown layout %d", c->layout);
    if (c->reserved != 0) return set_error(LPX_ERR_INVALID_ARG, "reserved must be 0");
    if (c->nt > (int64_t)1 << 40 || c->ns > (int64_t)1 << 40)
        return set_error(LPX_ERR_INVALID_ARG, "nt and ns must be below 2^40");
    if (c->nt == 0) return LPX_OK;
    if (!c->targets || !c->phi || (c->ns > 0 && !c->sources))
        return set_error(LPX_ERR_INVALID_ARG, "NULL targets, sources or phi");
    const bool aos = c->layout == LPX_ELEMENT_MAJOR;
    const uintptr_t mask = aos ? 15u : 3u;
    if ((reinterpret_cast<uintptr_t>(c->targets) & mask) ||
        (c->ns > 0 && (reinterpret_cast<uintptr_t>(c->sources) & mask)) ||
        (reinterpret_cast<uintptr_t>(c->phi) & 3u))
        return set_error(LPX_ERR_INVALID_ARG, aos ? "targets and sources must be 16-byte aligned"
                                                  : "misaligned pointer");
    const int64_t tbytes = c->nt * (aos ? 16 : 12), sbytes = c->ns * 16, pbytes = c->nt * 4;
    if (overlaps(c->phi, pbytes, c->targets, tbytes) ||
        overlaps(c->phi, pbytes, c->sources, sbytes))
        return set_error(LPX_ERR_ALIAS, "phi overlaps targets or sources");
    *noop = false;
    return LPX_OK;
}

}  // namespace lpx

using namespace lpx;

extern "C" {

lpx_status lpx_coulomb_validate(const lpx_coulomb_desc* c, const lpx_record* rec) {
    clear_error();
    try {
        bool noop;
        return validate_coulomb(c, rec, &noop);
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_coulomb(const lpx_coulomb_desc* c, const lpx_record* rec, void* stream) {
    clear_error();
    try {
        bool noop;
        lpx_status s = validate_coulomb(c, rec, &noop);
        if (s != LPX_OK || noop) return s;
        const lpx_record r = rec ? *rec : default_record(LPX_FP32);
        const int tile_s = 16 * r.tile_e, ilp = r.unroll;
        const bool stage = r.prefetch == 2;
        coul::Fn fn = c->layout == LPX_ELEMENT_MAJOR
                          ? coul::by_tile<LPX_ELEMENT_MAJOR>(tile_s, stage, ilp)
                          : coul::by_tile<LPX_DOF_MAJOR>(tile_s, stage, ilp);
        coul::Args a{c->targets, c->sources, c->phi, c->nt, c->ns};
        const int64_t grid = ceil_div(c->nt, (int64_t)coul::kThreads * ilp);
        if (grid > 0x7fffffff) return set_error(LPX_ERR_UNSUPPORTED, "too many targets");
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(coul::kThreads), 0, st, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return set_error(LPX_ERR_HIP, "Coulomb launch: %s", hipGetErrorString(e));
        return LPX_OK;
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

}  // extern "C"
