// Dense GEMM C = A B (row-major FP32 in and out), the contraction's
// degenerate case: the reduction sum(k, a[i,k]*b[k,j]) of the paper's
// sec. 2.1, Table 1's "sgemm" row.
//
// Tiling (split_iname of m, n and k; sec. 2.4.1): a work-group of four
// wave64s computes a TM x TN tile of C, each wave a (TM/2) x (TN/2) quarter
// made of 16 x 16 MFMA blocks.  The k loop runs over TK-deep slabs: the A
// slab (TM x TK) and the B slab (TK x TN, stored transposed as TN x TK) are
// staged in LDS in the operand precision (add_prefetch, sec. 2.4.4); the
// next slab is loaded from global memory into registers while the current
// one is multiplied.
//
// MFMA roles: the n index goes on the MFMA row axis, so each lane ends with
// four consecutive n of one row m and stores them as one 16-byte write.
#include <hip/hip_runtime.h>

#include "lpx_internal.h"

namespace lpx {
namespace gemm {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct GemmArgs {
    const float* __restrict__ A;
    const float* __restrict__ B;
    float* __restrict__ C;
    int64_t M, N, K, lda, ldb, ldc;
    int64_t tiles_n;  // ceil(N / TN)
    int vec_a, vec_b;  // lda / ldb multiples of 4: 16-byte row accesses
};

template <int PREC>
struct P;
template <>
struct P<LPX_FP32> {
    static constexpr int KSTEP = 4, KPL = 1, PLANES = 1, EB = 4;  // elem bytes
    static constexpr int PAD = 2;  // row stride = 2 (mod 4) floats
};
template <>
struct P<LPX_BF16> {
    static constexpr int KSTEP = 32, KPL = 8, PLANES = 1, EB = 2;
    static constexpr int PAD = 8;  // row stride = 16 (mod 64) bytes
};
template <>
struct P<LPX_BF16X3> {
    static constexpr int KSTEP = 32, KPL = 8, PLANES = 2, EB = 2;
    static constexpr int PAD = 8;
};

template <int PREC, int TM, int TN, int TK>
struct Geo {
    static constexpr int LD = TK + P<PREC>::PAD;              // LDS row stride
    static constexpr int A_ELEMS = TM * LD, B_ELEMS = TN * LD;  // per plane
    static constexpr int BYTES = (A_ELEMS + B_ELEMS) * P<PREC>::EB * P<PREC>::PLANES;
    static constexpr int A_CHUNKS = TM * TK / 4 / 256;  // float4 per thread
    static constexpr int B_CHUNKS = TN * TK / 4 / 256;
    static constexpr int BM = TM / 32, BN = TN / 32;    // 16x16 blocks per wave
};

template <int PREC>
__device__ __forceinline__ void put(unsigned char* plane0, int plane_elems, int idx, float v) {
    if constexpr (PREC == LPX_FP32) {
        reinterpret_cast<float*>(plane0)[idx] = v;
    } else {
        __bf16* p = reinterpret_cast<__bf16*>(plane0);
        const __bf16 h = (__bf16)v;
        p[idx] = h;
        if constexpr (PREC == LPX_BF16X3) p[plane_elems + idx] = (__bf16)(v - (float)h);
    }
}

// One 16-row operand fragment: rows r0 + lane%16 of a [rows][LD] plane,
// k-slots (lane/16)*KPL.. of step s.
template <int PREC>
struct Fr;
template <>
struct Fr<LPX_FP32> {
    float a;
};
template <>
struct Fr<LPX_BF16> {
    bf16x8 h;
};
template <>
struct Fr<LPX_BF16X3> {
    bf16x8 h, l;
};

template <int PREC, int LD, int PLANE>
__device__ __forceinline__ Fr<PREC> frag(const unsigned char* base, int r0, int s, int lane) {
    const int r = r0 + (lane & 15);
    const int k = s * P<PREC>::KSTEP + (lane >> 4) * P<PREC>::KPL;
    if constexpr (PREC == LPX_FP32) {
        return {reinterpret_cast<const float*>(base)[r * LD + k]};
    } else if constexpr (PREC == LPX_BF16) {
        return {*reinterpret_cast<const bf16x8*>(reinterpret_cast<const __bf16*>(base) + r * LD + k)};
    } else {
        const __bf16* p = reinterpret_cast<const __bf16*>(base);
        return {*reinterpret_cast<const bf16x8*>(p + r * LD + k),
                *reinterpret_cast<const bf16x8*>(p + PLANE + r * LD + k)};
    }
}

__device__ __forceinline__ f4 mma(const Fr<LPX_FP32>& a, const Fr<LPX_FP32>& b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a.a, b.a, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma(const Fr<LPX_BF16>& a, const Fr<LPX_BF16>& b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma(const Fr<LPX_BF16X3>& a, const Fr<LPX_BF16X3>& b, f4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
}

// Four consecutive floats of a row at column c, zero past `n`; one 16-byte
// load when rows are 16-byte aligned (vec) and all four are in range.
__device__ __forceinline__ f4 load4(const float* __restrict__ row, int64_t c, int64_t n,
                                    bool row_ok, bool vec) {
    if (vec && row_ok && c + 4 <= n) return *reinterpret_cast<const f4*>(row + c);
    f4 v = {0.f, 0.f, 0.f, 0.f};
    if (row_ok) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (c + q < n) v[q] = row[c + q];
    }
    return v;
}

template <int PREC, int TM, int TN, int TK>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    using G = Geo<PREC, TM, TN, TK>;
    constexpr int LD = G::LD;
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char* As = lds;
    unsigned char* Bs = lds + G::A_ELEMS * P<PREC>::EB * P<PREC>::PLANES;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m0 = (int64_t)(blockIdx.x / g.tiles_n) * TM;
    const int64_t n0 = (int64_t)(blockIdx.x % g.tiles_n) * TN;
    const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * (TN / 2);

    f4 acc[G::BN][G::BM];
#pragma unroll
    for (int bn = 0; bn < G::BN; ++bn)
#pragma unroll
        for (int bm = 0; bm < G::BM; ++bm) acc[bn][bm] = f4{0.f, 0.f, 0.f, 0.f};

    f4 ra[G::A_CHUNKS], rb[G::B_CHUNKS];
    // A slab: TM rows x TK columns, chunk c -> row c / (TK/4), column 4*(c % (TK/4)).
    // B slab: TK rows x TN columns, chunk c -> row c / (TN/4), column 4*(c % (TN/4)).
    auto load_slab = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < G::A_CHUNKS; ++q) {
            const int c = tid + 256 * q;
            const int r = c / (TK / 4), col = 4 * (c % (TK / 4));
            const int64_t m = m0 + r;
            ra[q] = load4(g.A + m * g.lda, k0 + col, g.K, m < g.M, g.vec_a);
        }
#pragma unroll
        for (int q = 0; q < G::B_CHUNKS; ++q) {
            const int c = tid + 256 * q;
            const int r = c / (TN / 4), col = 4 * (c % (TN / 4));
            const int64_t k = k0 + r;
            rb[q] = load4(g.B + k * g.ldb, n0 + col, g.N, k < g.K, g.vec_b);
        }
    };
    auto store_slab = [&]() {
#pragma unroll
        for (int q = 0; q < G::A_CHUNKS; ++q) {
            const int c = tid + 256 * q;
            const int r = c / (TK / 4), col = 4 * (c % (TK / 4));
#pragma unroll
            for (int t = 0; t < 4; ++t) put<PREC>(As, G::A_ELEMS, r * LD + col + t, ra[q][t]);
        }
#pragma unroll
        for (int q = 0; q < G::B_CHUNKS; ++q) {
            const int c = tid + 256 * q;
            const int r = c / (TN / 4), col = 4 * (c % (TN / 4));
#pragma unroll
            for (int t = 0; t < 4; ++t) put<PREC>(Bs, G::B_ELEMS, (col + t) * LD + r, rb[q][t]);
        }
    };

    const int64_t nk = (g.K + TK - 1) / TK;
    load_slab(0);
    for (int64_t kt = 0; kt < nk; ++kt) {
        __syncthreads();  // the previous slab is no longer read
        store_slab();
        __syncthreads();
        if (kt + 1 < nk) load_slab((kt + 1) * TK);  // in flight during the MFMAs
#pragma unroll
        for (int s = 0; s < TK / P<PREC>::KSTEP; ++s) {
            Fr<PREC> fa[G::BM];
#pragma unroll
            for (int bm = 0; bm < G::BM; ++bm)
                fa[bm] = frag<PREC, LD, G::A_ELEMS>(As, wm + 16 * bm, s, lane);
#pragma unroll
            for (int bn = 0; bn < G::BN; ++bn) {
                const Fr<PREC> fb = frag<PREC, LD, G::B_ELEMS>(Bs, wn + 16 * bn, s, lane);
#pragma unroll
                for (int bm = 0; bm < G::BM; ++bm) acc[bn][bm] = mma(fb, fa[bm], acc[bn][bm]);
            }
        }
    }

    // acc[bn][bm]: lane holds C[m][n .. n+3], m = wm + 16 bm + lane%16,
    // n = wn + 16 bn + 4 (lane/16).
    const bool vec = (g.ldc % 4) == 0;
#pragma unroll
    for (int bn = 0; bn < G::BN; ++bn)
#pragma unroll
        for (int bm = 0; bm < G::BM; ++bm) {
            const int64_t m = m0 + wm + 16 * bm + (lane & 15);
            const int64_t n = n0 + wn + 16 * bn + 4 * (lane >> 4);
            if (m >= g.M || n >= g.N) continue;
            float* dst = g.C + m * g.ldc + n;
            if (vec && n + 4 <= g.N) {
                *reinterpret_cast<f4*>(dst) = acc[bn][bm];
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (n + r < g.N) dst[r] = acc[bn][bm][r];
            }
        }
}

using GemmFn = void (*)(GemmArgs);

template <int PREC>
GemmFn pick(int tm, int tn, int tk, int* lds) {
#define LPX_GEMM_CASE(TM_, TN_, TK_)                                 \
    if (tm == TM_ && tn == TN_ && tk == TK_) {                       \
        *lds = Geo<PREC, TM_, TN_, TK_>::BYTES;                      \
        return &gemm_kernel<PREC, TM_, TN_, TK_>;                    \
    }
    LPX_GEMM_CASE(64, 64, 32)
    LPX_GEMM_CASE(64, 64, 64)
    LPX_GEMM_CASE(128, 128, 32)
    LPX_GEMM_CASE(128, 128, 64)
    LPX_GEMM_CASE(128, 64, 32)
    LPX_GEMM_CASE(64, 128, 32)
    if constexpr (PREC != LPX_BF16X3) {
        LPX_GEMM_CASE(256, 128, 32)
        LPX_GEMM_CASE(128, 256, 32)
        LPX_GEMM_CASE(256, 256, 32)
    }
#undef LPX_GEMM_CASE
    return nullptr;
}

}  // namespace gemm

bool gemm_split_tiling(int precision, int tm, int tn, int tk);

lpx_status gemm_tiles(const lpx_record& r, int* tm, int* tn, int* tk) {
    // default: 128 x 128 x 64 for the reduced precisions (the pre-split
    // path), 128 x 128 x 32 for fp32
    *tm = r.gemm_tm ? r.gemm_tm : 128;
    *tn = r.gemm_tn ? r.gemm_tn : 128;
    *tk = r.gemm_tk ? r.gemm_tk : (r.precision == LPX_FP32 ? 32 : 64);
    if (gemm_split_tiling(r.precision, *tm, *tn, *tk)) return LPX_OK;
    int lds = 0;
    void* fn = nullptr;
    switch (r.precision) {
        case LPX_FP32: fn = (void*)gemm::pick<LPX_FP32>(*tm, *tn, *tk, &lds); break;
        case LPX_BF16: fn = (void*)gemm::pick<LPX_BF16>(*tm, *tn, *tk, &lds); break;
        default: fn = (void*)gemm::pick<LPX_BF16X3>(*tm, *tn, *tk, &lds); break;
    }
    if (!fn)
        return set_error(LPX_ERR_UNSUPPORTED,
                         "GEMM tile %dx%dx%d is not built for this precision (built: 64x64x32, "
                         "64x64x64, 128x128x32, 128x128x64, 128x64x32, 64x128x32; fp32/bf16 also "
                         "256x128x32, 128x256x32, 256x256x32; bf16 256x256x64, 256x128x64; "
                         "bf16x3 256x256x32, 256x128x32 (pre-split))",
                         *tm, *tn, *tk);
    return LPX_OK;
}

lpx_status launch_gemm_split(const lpx_gemm_desc& d, int precision, int tm, int tn, int tk,
                             void* stream);

lpx_status launch_gemm(const lpx_gemm_desc& d, const lpx_record& r, void* stream) {
    int tm, tn, tk, lds = 0;
    lpx_status s = gemm_tiles(r, &tm, &tn, &tk);
    if (s != LPX_OK) return s;
    // bf16x3 default: 256 x 256 x 32 once C has a 256 x 256 tile per compute
    // unit (three MFMAs per product keep the single wave per SIMD busy; below
    // that the 128 x 128 tiles fill the chip better)
    if (r.precision == LPX_BF16X3 && !r.gemm_tm && !r.gemm_tn && !r.gemm_tk &&
        ceil_div(d.M, 256) * ceil_div(d.N, 256) >= 256)
        tm = 256, tn = 256, tk = 32;
    // bf16 / bf16x3 at 128 x 128 x 64 and the 256-row tilings: operands split
    // once into bf16 planes, then the direct-to-LDS kernel (nothing to split
    // when K == 0: the general kernel writes the zeros)
    const bool split = gemm_split_tiling(r.precision, tm, tn, tk);
    if (split && d.K > 0) return launch_gemm_split(d, r.precision, tm, tn, tk, stream);
    if (split) tm = 128, tn = 128, tk = 64;
    gemm::GemmFn fn = nullptr;
    switch (r.precision) {
        case LPX_FP32: fn = gemm::pick<LPX_FP32>(tm, tn, tk, &lds); break;
        case LPX_BF16: fn = gemm::pick<LPX_BF16>(tm, tn, tk, &lds); break;
        default: fn = gemm::pick<LPX_BF16X3>(tm, tn, tk, &lds); break;
    }
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess)
            return set_error(LPX_ERR_HIP, "hipFuncSetAttribute: %s", hipGetErrorString(e));
    }
    gemm::GemmArgs a;
    a.A = d.A;
    a.B = d.B;
    a.C = d.C;
    a.M = d.M;
    a.N = d.N;
    a.K = d.K;
    a.lda = d.lda;
    a.ldb = d.ldb;
    a.ldc = d.ldc;
    a.tiles_n = ceil_div(d.N, tn);
    a.vec_a = (d.lda % 4) == 0;
    a.vec_b = (d.ldb % 4) == 0;
    const int64_t grid = ceil_div(d.M, tm) * a.tiles_n;
    if (grid > 0x7fffffff) return set_error(LPX_ERR_UNSUPPORTED, "GEMM grid too large");
    void* args[] = {&a};
    hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)grid),
                                   dim3(256), args, (size_t)lds,
                                   reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return set_error(LPX_ERR_HIP, "GEMM launch: %s", hipGetErrorString(e));
    return LPX_OK;
}

}  // namespace lpx
