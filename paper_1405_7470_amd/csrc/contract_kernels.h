// Contraction kernel family  out[k,e,i] = sum_j D[k][i][j] u[e][j]  for gfx950.
//
// One template, instantiated once per transformation record:
//
//   PREC      FP32 (v_mfma_f32_16x16x4_f32), BF16 or BF16X3
//             (v_mfma_f32_16x16x32_bf16; bf16x3 = three products per step)
//   LAYOUT    element-major or DOF-major storage of u and out (the paper's
//             array-axis tags, sec. 2.4.3)
//   NTMAX     compiled bound on the number of 16-row i-blocks (2, 4, 8)
//   TILE_E    split_iname(e, TILE_E), outer index -> work-group (sec. 2.4.1)
//   PREFETCH  add_prefetch (sec. 2.4.4), one bit per array: bit 0 stages all
//             of D in LDS (once per work-group), bit 1 stages each u tile,
//             bit 2 keeps D in registers, bit 3 stages each output tile
//   UNROLL    split of the MFMA k-step loop with the inner part unrolled
//             (tag "unr", sec. 2.4.2)
//
// Row blocks.  The K operators are stacked into one (K*Np) x Np matrix
// (D[k][i][j] is row k*Np + i of D viewed as [K*Np][Np]) and cut into
// nrb = ceil(K*Np/16) blocks of 16 rows: one MFMA row block covers rows of
// consecutive operators, so only the last block is padded (K = 3, Np = 56:
// 11 blocks instead of 12 per-operator ones).  Each output keeps the same
// reduction over j, whichever block its row lands in.
//
// Work decomposition.  A work-group (4 wave64s per 16 elements of the
// tile) walks the element tiles
// tile = blockIdx.x, blockIdx.x + gridDim.x, ... (grid sized to the
// resident capacity, so LDS-staged D is loaded once per work-group).
// Without the u bit, each wave streams its u fragments from global memory
// straight into registers and needs no work-group barrier per tile.  A tile
// of TILE_E elements is split into 16-element blocks; each block's K*nt
// (operator, i-block) pairs are spread over its 4 waves.  A wave owns a
// set of pairs and, for one 16-element block, accumulates
//     C_pair[16 x 16] += A[16 x kstep] * B[kstep x 16]
// over the k-steps of j.  The two operands are a D fragment (16 rows of
// D[k] for the pair's i-block) and a u fragment (the 16 elements of the
// block).  Element-major puts i on the MFMA row axis, so each lane ends
// with 4 consecutive i of one element (one 16-byte store); DOF-major puts
// e on the row axis, so each lane ends with 4 consecutive e of one i.
//
// MFMA operand layout (16x16xKSTEP, both A and B): lane l supplies row (or
// column) l % 16 and the k-slots (l / 16) * KPL ... + KPL - 1 of the step,
// KPL = 1 (fp32) or 8 (bf16).  The product pairs A and B values of the same
// lane-group/slot, so any mapping of j onto (step, group, slot) is correct
// as long as both operands use it.  bf16: j = step*32 + group*8 + slot.
// fp32: steps come in quads of four (16 columns); step 4Q+m of quad Q gives
// group g the column j = 16Q + 4g + m, so a lane's four values of a quad
// are consecutive in memory and arrive in one 16-byte read.  Steps after
// the last whole quad use j = 4*step + g.
// The 16x16 result: lane l, register r holds row 4*(l/16) + r, column l%16.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lpx_internal.h"

namespace lpx {
namespace kern {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct ContractArgs {
    const float* __restrict__ D;
    const float* __restrict__ u;
    float* __restrict__ out;
    // D in MFMA operand order in global memory, written by arrange_d_kernel
    // for kernels that read D from memory (prefetch bits 0 and 2 clear)
    const unsigned char* __restrict__ Darr;
    int64_t E;
    int64_t ntiles;
    int K, Np, nt, nsteps, ldu;
    int nrb;     // stacked row blocks: ceil(K * Np / 16)
    Divider np_div;  // stacked row R -> operator R / Np
    int ldo;     // staged output slot stride (floats), prefetch bit 3
    // dG volume term (EPI = 1): geometric factors, and the float offset of
    // the tile's copy of them inside each staged output slot
    const float* __restrict__ G;
    int ldo_g;
    int np_vec;  // Np % 4 == 0: 16-byte row accesses are aligned
    int e_vec;   // E % 4 == 0
    int stream_out;  // large outputs: streaming (non-temporal) stores, see store_stream
    int blocked;     // record order 1: work-group b takes one contiguous range of tiles
};

// Operator index of stacked row R (0 <= R < 2^31).
__device__ __forceinline__ int row_op(const ContractArgs& a, int R) {
    return (int)(((uint64_t)(uint32_t)R * a.np_div.m) >> a.np_div.sh);
}

template <int PREC>
struct Frag;
template <>
struct Frag<LPX_FP32> {
    float a;
};
template <>
struct Frag<LPX_BF16> {
    bf16x8 h;
};
template <>
struct Frag<LPX_BF16X3> {
    bf16x8 h, l;
};

template <int PREC>
struct Traits {
    static constexpr int KSTEP = 32;  // reduction length of one MFMA
    static constexpr int KPL = 8;     // k-slots per lane
};
template <>
struct Traits<LPX_FP32> {
    static constexpr int KSTEP = 4;
    static constexpr int KPL = 1;
};

// Column j of lane group g at fp32 step s (nquad_steps = 4 * whole quads).
__device__ __forceinline__ int fp32_col(int s, int g, int nquad_steps) {
    return s < nquad_steps ? 16 * (s >> 2) + 4 * g + (s & 3) : 4 * s + g;
}

// ------------------------------------------------------------ conversions
__device__ __forceinline__ Frag<LPX_FP32> make_frag_fp32(float v) { return {v}; }

template <int PREC>
__device__ __forceinline__ Frag<PREC> make_frag8(const float (&v)[8]);

template <>
__device__ __forceinline__ Frag<LPX_BF16> make_frag8<LPX_BF16>(const float (&v)[8]) {
    Frag<LPX_BF16> f;
#pragma unroll
    for (int t = 0; t < 8; ++t) f.h[t] = (__bf16)v[t];  // round to nearest even
    return f;
}

template <>
__device__ __forceinline__ Frag<LPX_BF16X3> make_frag8<LPX_BF16X3>(const float (&v)[8]) {
    Frag<LPX_BF16X3> f;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        __bf16 h = (__bf16)v[t];
        f.h[t] = h;
        f.l[t] = (__bf16)(v[t] - (float)h);  // the difference is exact in fp32
    }
    return f;
}

// ------------------------------------------------------------------ MFMA
__device__ __forceinline__ f4 mma(const Frag<LPX_FP32>& a, const Frag<LPX_FP32>& b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a.a, b.a, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma(const Frag<LPX_BF16>& a, const Frag<LPX_BF16>& b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
}
// bf16x3: the two correction products first, then hi*hi.
__device__ __forceinline__ f4 mma(const Frag<LPX_BF16X3>& a, const Frag<LPX_BF16X3>& b,
                                  f4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
}

// ------------------------------------------------------- global fragments
// Loads here never sit behind a per-lane branch: out-of-range lanes read a
// clamped in-bounds address and the value is replaced by zero with a select
// where it is consumed.  (A divergent branch around a load makes the
// compiler wait for that load at the join, serialising every load.)

// Eight consecutive values row[j0 .. j0+8), zero at columns >= n (n >= 1).
// vec: the row start is 16-byte aligned and n % 4 == 0, so each half is
// either wholly inside or wholly outside the row.
__device__ __forceinline__ void load_row8(const float* __restrict__ row, int j0, int n,
                                          bool vec, float (&v)[8]) {
    if (vec) {  // uniform
        const int ja = j0 < n - 4 ? j0 : n - 4;
        const int jb = j0 + 4 < n - 4 ? j0 + 4 : n - 4;
        const f4 a = *reinterpret_cast<const f4*>(row + ja);
        const f4 b = *reinterpret_cast<const f4*>(row + jb);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            v[t] = j0 + t < n ? a[t] : 0.0f;
            v[t + 4] = j0 + 4 + t < n ? b[t] : 0.0f;
        }
    } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int j = j0 + t < n ? j0 + t : n - 1;
            const float x = row[j];
            v[t] = j0 + t < n ? x : 0.0f;
        }
    }
}

// D fragment of row block p, step s, read from global memory.
template <int PREC>
__device__ __forceinline__ Frag<PREC> d_frag_global(const ContractArgs& a, int p, int s,
                                                    int lane) {
    const int rows = a.K * a.Np;
    const int R = 16 * p + (lane & 15);
    const float* row = a.D + (int64_t)(R < rows ? R : rows - 1) * a.Np;
    if constexpr (PREC == LPX_FP32) {
        const int j0 = fp32_col(s, lane >> 4, a.nsteps & ~3);
        const float x = row[j0 < a.Np ? j0 : a.Np - 1];
        return make_frag_fp32(R < rows && j0 < a.Np ? x : 0.0f);
    } else {
        const int j0 = s * Traits<PREC>::KSTEP + (lane >> 4) * Traits<PREC>::KPL;
        float v[8];
        load_row8(row, j0, a.Np, a.np_vec, v);
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = R < rows ? v[q] : 0.0f;
        return make_frag8<PREC>(v);
    }
}

// u fragment of the 16-element block starting at eb0, step s, from global.
template <int PREC, int LAYOUT>
__device__ __forceinline__ Frag<PREC> u_frag_global(const ContractArgs& a, int64_t eb0,
                                                    int s, int lane) {
    const int64_t e = eb0 + (lane & 15);
    const bool ev = e < a.E;
    const int64_t ec = ev ? e : a.E - 1;
    if constexpr (PREC == LPX_FP32) {
        const int j0 = fp32_col(s, lane >> 4, a.nsteps & ~3);
        const int jc = j0 < a.Np ? j0 : a.Np - 1;
        const float x = LAYOUT == LPX_ELEMENT_MAJOR ? a.u[ec * a.Np + jc] : a.u[(int64_t)jc * a.E + ec];
        return make_frag_fp32(ev && j0 < a.Np ? x : 0.0f);
    } else {
        const int j0 = s * Traits<PREC>::KSTEP + (lane >> 4) * Traits<PREC>::KPL;
        float v[8];
        if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
            load_row8(a.u + ec * a.Np, j0, a.Np, a.np_vec, v);
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int j = j0 + t < a.Np ? j0 + t : a.Np - 1;
                const float x = a.u[(int64_t)j * a.E + ec];
                v[t] = j0 + t < a.Np ? x : 0.0f;
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = ev ? v[t] : 0.0f;
        return make_frag8<PREC>(v);
    }
}

// fp32 quads from global memory: the lane's four values of quad Q.
// Four consecutive values row[j0 .. j0+4), zero at columns >= n (n >= 1,
// j0 % 4 == 0).  vec: 16-byte aligned row start and n % 4 == 0.
__device__ __forceinline__ f4 load_row4(const float* __restrict__ row, int j0, int n,
                                        bool vec) {
    f4 v;
    if (vec) {  // uniform
        const f4 x = *reinterpret_cast<const f4*>(row + (j0 < n ? j0 : n - 4));
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = j0 + t < n ? x[t] : 0.0f;
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float x = row[j0 + t < n ? j0 + t : n - 1];
            v[t] = j0 + t < n ? x : 0.0f;
        }
    }
    return v;
}

__device__ __forceinline__ f4 d_quad_global(const ContractArgs& a, int p, int Q, int lane) {
    const int rows = a.K * a.Np;
    const int R = 16 * p + (lane & 15);
    const f4 v = load_row4(a.D + (int64_t)(R < rows ? R : rows - 1) * a.Np,
                           16 * Q + 4 * (lane >> 4), a.Np, a.np_vec);
    const f4 z = {0.0f, 0.0f, 0.0f, 0.0f};
    return R < rows ? v : z;
}

template <int LAYOUT>
__device__ __forceinline__ f4 u_quad_global(const ContractArgs& a, int64_t eb0, int Q,
                                            int lane) {
    const int64_t e = eb0 + (lane & 15);
    const bool ev = e < a.E;
    const int64_t ec = ev ? e : a.E - 1;
    const int j0 = 16 * Q + 4 * (lane >> 4);
    f4 v;
    if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
        v = load_row4(a.u + ec * a.Np, j0, a.Np, a.np_vec);
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int j = j0 + t < a.Np ? j0 + t : a.Np - 1;
            const float x = a.u[(int64_t)j * a.E + ec];
            v[t] = j0 + t < a.Np ? x : 0.0f;
        }
    }
    const f4 z = {0.0f, 0.0f, 0.0f, 0.0f};
    return ev ? v : z;
}

// ------------------------------------------------------------ LDS layout
// [D fragments, operand order: ((k*nt + t)*nsteps + s)*64 + lane]
//   fp32: float; bf16: 16-byte hi plane; bf16x3: hi plane then lo plane.
//   fp32 quads are lane-major inside their 4*64-float block: step 4Q+m of
//   pair p, lane l sits at (p*nsteps + 4Q)*64 + 4l + m (one 16-byte read
//   per lane and quad); the steps after the last quad keep operand order.
// [u ring: four slots of ldu floats, raw FP32 copies of u tiles]
// [output ring (prefetch bit 3): two slots of ldo floats]
template <int PREC>
struct Lds {
    static constexpr int DFRAG_BYTES = PREC == LPX_FP32 ? 4 : 16;  // per plane
    static constexpr int PLANES = PREC == LPX_BF16X3 ? 2 : 1;
    static constexpr int UELEM_BYTES = PREC == LPX_FP32 ? 4 : 2;
};

// Element idx of an array of T at `base`: in LDS, or (GLOBAL) in global
// memory.  The global case reads through a global-address-space pointer, so
// the load is a global load even where the compiler cannot trace the
// pointer to a kernel argument (the batch reads it from its descriptor
// table; a generic pointer there gives flat loads, which also count against
// the LDS wait counter).
template <class T, bool GLOBAL>
__device__ __forceinline__ T load_elem(const unsigned char* base, int64_t idx) {
    if constexpr (GLOBAL) {
        typedef __attribute__((address_space(1))) const T GT;
        return ((GT*)base)[idx];
    } else {
        return reinterpret_cast<const T*>(base)[idx];
    }
}

// D fragments in MFMA operand order: staged in LDS, or (GLOBAL) the same
// arrangement in global memory.
template <int PREC, bool GLOBAL = false>
__device__ __forceinline__ Frag<PREC> d_frag_lds(const unsigned char* lds, int64_t nfrag,
                                                 int idx) {
    if constexpr (PREC == LPX_FP32) {
        return {load_elem<float, GLOBAL>(lds, idx)};
    } else if constexpr (PREC == LPX_BF16) {
        return {load_elem<bf16x8, GLOBAL>(lds, idx)};
    } else {
        return {load_elem<bf16x8, GLOBAL>(lds, idx), load_elem<bf16x8, GLOBAL>(lds, nfrag + idx)};
    }
}

template <bool GLOBAL = false>
__device__ __forceinline__ f4 d_quad_lds(const unsigned char* lds, int p, int Q, int nsteps,
                                         int lane) {
    return load_elem<f4, GLOBAL>(lds, (p * nsteps + 4 * Q) * 16 + lane);
}

template <int PREC>
__device__ __forceinline__ void d_frag_store_lds(unsigned char* lds, int64_t nfrag, int idx,
                                                 const Frag<PREC>& f) {
    if constexpr (PREC == LPX_FP32) {
        reinterpret_cast<float*>(lds)[idx] = f.a;
    } else if constexpr (PREC == LPX_BF16) {
        reinterpret_cast<bf16x8*>(lds)[idx] = f.h;
    } else {
        bf16x8* p = reinterpret_cast<bf16x8*>(lds);
        p[idx] = f.h;
        p[nfrag + idx] = f.l;
    }
}

// ---------------------------------------------------- staged u tiles
// A staged u tile is a raw copy of the tile's bytes in global memory, in a
// four-slot LDS ring (three tiles in flight while the fourth is read):
//   element-major: the contiguous run u[e0 .. e0+nvalid)[0 .. Np), so
//                  element r, column j sits at r*Np + j;
//   DOF-major:     the Np row segments u[j][e0 .. e0+TILE_E), so column j,
//                  element r sits at j*TILE_E + r.
// A slot has slack past the tile so that reads of padding columns
// (j >= Np, up to the next multiple of 32) stay inside it; those values are
// replaced by zero with a select, never multiplied.  Compute waves convert
// what they read to the operand precision.
// MASK: zero the columns j >= Np.  Without it the caller guarantees that
// every column it uses is below Np (the values read for other columns may
// belong to the next element or to the slot's slack).
// DOF-major tiles of 64 elements (one 256-byte row per column j, all of
// the LDS banks) are stored with the 16-byte chunks of each row permuted:
// element r of column j sits at r ^ (16 * ((j >> 2) & 3)).  The four lane
// groups of an MFMA operand read columns four apart (j = 16Q + 4g + t), which
// unpermuted start at the same bank; permuted, group g reads the quarter of
// the banks that r ^ 16g selects.  The loader writes each chunk to its
// permuted place by choosing which global chunk each lane fetches.
template <int LAYOUT, int TILE_E>
__device__ __forceinline__ int dm_swz(int j) {
    return (LAYOUT == LPX_DOF_MAJOR && TILE_E == 64) ? ((j >> 2) & 3) << 4 : 0;
}

template <int PREC, int LAYOUT, int TILE_E, bool MASK = true>
__device__ __forceinline__ Frag<PREC> u_frag_lds(const float* ut, int Np, bool np_vec, int row0,
                                                 int s, int nquad_steps, int lane) {
    const int r = row0 + (lane & 15);
    if constexpr (PREC == LPX_FP32) {
        const int j0 = fp32_col(s, lane >> 4, nquad_steps);
        const int jc = j0 < Np ? j0 : Np - 1;  // callers may read steps past the last
        const float x = LAYOUT == LPX_ELEMENT_MAJOR
                            ? ut[r * Np + jc]
                            : ut[jc * TILE_E + (r ^ dm_swz<LAYOUT, TILE_E>(jc))];
        if constexpr (MASK) return {j0 < Np ? x : 0.0f};
        return {x};
    } else {
        const int j0 = s * Traits<PREC>::KSTEP + (lane >> 4) * Traits<PREC>::KPL;
        float v[8];
        if (LAYOUT == LPX_ELEMENT_MAJOR && np_vec) {  // 16-byte aligned rows
            const f4 a = *reinterpret_cast<const f4*>(ut + r * Np + j0);
            const f4 b = *reinterpret_cast<const f4*>(ut + r * Np + j0 + 4);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                v[t] = a[t];
                v[t + 4] = b[t];
            }
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t)
                v[t] = LAYOUT == LPX_ELEMENT_MAJOR
                           ? ut[r * Np + j0 + t]
                           : ut[(j0 + t) * TILE_E + (r ^ dm_swz<LAYOUT, TILE_E>(j0 + t))];
        }
        if constexpr (MASK) {
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = j0 + t < Np ? v[t] : 0.0f;
        }
        return make_frag8<PREC>(v);
    }
}

// fp32 quad Q of the staged tile (see u_frag_lds for the layout and MASK).
template <int LAYOUT, int TILE_E, bool MASK = true>
__device__ __forceinline__ f4 u_quad_lds(const float* ut, int Np, bool np_vec, int row0, int Q,
                                         int lane) {
    const int r = row0 + (lane & 15);
    const int j0 = 16 * Q + 4 * (lane >> 4);
    f4 v;
    if (LAYOUT == LPX_ELEMENT_MAJOR && np_vec) {  // 16-byte aligned rows
        v = *reinterpret_cast<const f4*>(ut + r * Np + j0);
    } else if constexpr (LAYOUT == LPX_DOF_MAJOR) {
        // columns j0 .. j0+3 share (j >> 2) & 3 = lane group: one permuted slot
        const float* p = ut + j0 * TILE_E + (r ^ dm_swz<LAYOUT, TILE_E>(j0));
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = p[t * TILE_E];
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = ut[r * Np + j0 + t];
    }
    if constexpr (MASK) {
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = j0 + t < Np ? v[t] : 0.0f;
    }
    return v;
}

// Loader waves fill the u ring with direct global-to-LDS loads
// (global_load_lds: the data goes to LDS without passing through
// registers, each lane's 4 or 16 bytes at base + lane * size).  A tile is
// a raw copy of its bytes in global memory, cut into 16-byte chunks; chunk
// c sits at slot byte 16c.  Loader wave lw (of NLW) loads chunks
// c = lane + 64 * (lw * PER_LANE + q), q < PER_LANE.  Chunks past the tile are
// clamped to its last chunk (the duplicates land in the slot's slack and
// are never read), so every regular tile costs exactly PER_LANE load
// instructions per loader wave and the loader can wait for one tile with a
// compile-time vmcnt while later tiles are still in flight.
//   element-major: chunk c = floats 4c..4c+3 of the run of nvalid*Np floats;
//   DOF-major:     chunk c = row j = c / (TILE_E/4), columns
//                  4*(c % (TILE_E/4)) .. +3 (64-element tiles: the columns
//                  of the chunk that belongs at slot chunk c under dm_swz).
// A tile whose chunks are not all whole 16-byte aligned runs (the last
// element-major tile when nvalid*Np % 4 != 0; every DOF-major tile when
// E % 4 != 0) is loaded with 4-byte loads instead (4*PER_LANE
// instructions), and is waited for with vmcnt(0).
template <int TILE_E, int NTMAX, int NLW>
struct Loader {
    static constexpr int PER_LANE = loader_per_lane(TILE_E, NTMAX, NLW);
};

typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ void dma16(const float* g, float* lds_base) {
    __builtin_amdgcn_global_load_lds(static_cast<const void*>(g),
                                     (lds_void*)(lds_base), 16, 0, 0);
}
__device__ __forceinline__ void dma4(const float* g, float* lds_base) {
    __builtin_amdgcn_global_load_lds(static_cast<const void*>(g),
                                     (lds_void*)(lds_base), 4, 0, 0);
}

// s_waitcnt immediate that waits until at most n vector-memory operations
// of this wave are outstanding (other counters untouched).
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// Issues the loads of one tile into `slot`; returns true for a regular
// tile (exactly PER_LANE 16-byte loads from this wave).
template <int LAYOUT, int TILE_E, int NTMAX, int NLW>
__device__ __forceinline__ bool loader_issue(const ContractArgs& a, float* slot, int64_t e0,
                                             int nvalid, int lw, int lane) {
    constexpr int PL = Loader<TILE_E, NTMAX, NLW>::PER_LANE;
    if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
        const float* src = a.u + e0 * a.Np;  // 16-byte aligned: e0 % 16 == 0
        const int nflat = nvalid * a.Np;
        if (nflat % 4 == 0) {  // uniform
            const int nch = nflat / 4;
#pragma unroll
            for (int q = 0; q < PL; ++q) {
                const int w = lw * PL + q;
                const int c = lane + 64 * w;
                dma16(src + 4 * (c < nch ? c : nch - 1), slot + 256 * w);
            }
            return true;
        }
#pragma unroll
        for (int q = 0; q < 4 * PL; ++q) {
            const int w = lw * 4 * PL + q;
            const int f = lane + 64 * w;
            dma4(src + (f < nflat ? f : nflat - 1), slot + 64 * w);
        }
        return false;
    } else {
        // 64 lanes cover whole rows (CPR and TILE_E divide 64), so lane l of
        // instruction w reads row  l / CPR + w * (64 / CPR)  at a column that
        // does not depend on w: one base address per lane plus a uniform
        // row stride per instruction.
        // With 64-element tiles the slot position of a lane's chunk is fixed
        // and the permutation (dm_swz) picks the element chunk it fetches:
        // row j = lane / 16 + 4w has (j >> 2) & 3 = w & 3 (16-byte loads),
        // row j = w (4-byte loads).
        constexpr int CPR = TILE_E / 4;
        if (a.e_vec) {  // uniform: E % 4 == 0, so nvalid % 4 == 0 and rows are aligned
#pragma unroll
            for (int q = 0; q < PL; ++q) {
                const int w = lw * PL + q;
                int col = 4 * (lane % CPR);
                if constexpr (TILE_E == 64) col ^= (w & 3) << 4;
                col = col < nvalid ? col : nvalid - 4;  // columns >= nvalid are never used
                int j = lane / CPR + w * (64 / CPR);
                j = j < a.Np ? j : a.Np - 1;  // rows past Np land in the slot's slack
                dma16(a.u + e0 + col + (int64_t)j * a.E, slot + 256 * w);
            }
            return true;
        }
#pragma unroll
        for (int q = 0; q < 4 * PL; ++q) {
            const int w = lw * 4 * PL + q;
            int r = lane % TILE_E;
            if constexpr (TILE_E == 64) r ^= ((w >> 2) & 3) << 4;
            r = r < nvalid ? r : nvalid - 1;
            int j = lane / TILE_E + w * (64 / TILE_E);
            j = j < a.Np ? j : a.Np - 1;
            dma4(a.u + e0 + r + (int64_t)j * a.E, slot + 64 * w);
        }
        return false;
    }
}

// Loader-wave loop, shared by the contraction and batch kernels.  issue(n)
// starts the loads of the work-group's n-th tile into u slot n & 3 and
// returns whether the tile was regular (PL 16-byte loads).  Three tiles are
// in flight: in iteration n the loader starts tile n+3 (its slot was read by
// the compute waves in iteration n-1), then waits until tile n+1 has landed;
// one barrier per iteration, `niter` iterations after a prologue barrier.
// The waits and barriers are explicit: a loader wave touches no other LDS.
template <int PL, typename Issue>
__device__ __forceinline__ void loader_loop(int64_t nmine, int64_t niter, Issue&& issue) {
    unsigned regular = 0xf;  // bit s: the tile in slot s was regular
    auto start = [&](int64_t n) {
        const bool r = issue(n);
        regular = (regular & ~(1u << (n & 3))) | ((unsigned)r << (n & 3));
    };
    // Wait for tile m: the tiles after it that are in flight must all be
    // regular for a partial wait; otherwise wait for everything.
    auto wait_for = [&](int64_t m) {
        const int64_t later = (nmine - 1 - m) < 2 ? (nmine - 1 - m) : 2;
        const bool reg = (later < 1 || ((regular >> ((m + 1) & 3)) & 1)) &&
                         (later < 2 || ((regular >> ((m + 2) & 3)) & 1));
        if (reg && later == 2)
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(2 * PL));
        else if (reg && later == 1)
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(PL));
        else
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    };
    for (int64_t n = 0; n < 3 && n < nmine; ++n) start(n);
    if (nmine > 0) wait_for(0);
    __builtin_amdgcn_s_barrier();
    for (int64_t n = 0; n < niter; ++n) {
        if (n + 3 < nmine) start(n + 3);
        if (n + 1 < nmine) wait_for(n + 1);
        __builtin_amdgcn_s_barrier();
    }
}

// ------------------------------------------------------ building blocks
// D in MFMA operand order, converted to the operand precision, written to
// LDS by the NTHREADS threads of a work-group (caller adds the barrier).
template <int PREC, int NTHREADS>
__device__ __forceinline__ void stage_d(const ContractArgs& a, unsigned char* lds, int tid) {
    // Fragments are built in batches of U per thread so that U loads are in
    // flight together (D is small and read from L2 after the first touch).
    constexpr int U = PREC == LPX_FP32 ? 8 : 4;
    const int64_t nfrag = (int64_t)a.nrb * a.nsteps * 64;
    for (int64_t base = 0; base < nfrag; base += (int64_t)NTHREADS * U) {
        Frag<PREC> f[U];
#pragma unroll
        for (int b = 0; b < U; ++b) {
            int64_t idx = base + tid + (int64_t)NTHREADS * b;
            idx = idx < nfrag ? idx : nfrag - 1;  // clamped: the duplicate is not stored
            const int rest = (int)(idx >> 6);
            const int sb = rest % a.nsteps;  // 64-float block of the pair
            const int p = rest / a.nsteps;
            int l = (int)(idx & 63), s = sb;
            if (PREC == LPX_FP32 && sb < (a.nsteps & ~3)) {  // lane-major quad block
                const int w = (sb & 3) * 64 + l;
                l = w >> 2;
                s = (sb & ~3) + (w & 3);
            }
            f[b] = d_frag_global<PREC>(a, p, s, l);
        }
#pragma unroll
        for (int b = 0; b < U; ++b) {
            const int64_t idx = base + tid + (int64_t)NTHREADS * b;
            if (idx < nfrag) d_frag_store_lds<PREC>(lds, nfrag, (int)idx, f[b]);
        }
    }
}

// The same arrangement written to global memory once per call, for kernels
// that read D from memory: a wave's D loads are then lane-contiguous 16-byte
// (FP32 quads, bf16 planes) or 4-byte runs instead of 16 rows of 64 bytes.
constexpr int kArrangeThreads = 256, kArrangeBlocks = 64;
template <int PREC>
__global__ __launch_bounds__(kArrangeThreads) void arrange_d_kernel(ContractArgs a,
                                                                    unsigned char* dst) {
    stage_d<PREC, kArrangeThreads * kArrangeBlocks>(a, dst,
                                                    blockIdx.x * kArrangeThreads + threadIdx.x);
}

// Streaming store of 16 bytes (the non-temporal hint: the line is written
// through without being kept in the caches).  Used where every store
// instruction writes whole contiguous runs (the store waves' copy-out, 1 KiB
// per instruction) and for the DOF-major direct stores; measured on MI355X at
// K=3, Np=56, E=2^20, one launch timed alone: bf16x3 staged-output kernels
// 187 -> 142-148 us (element-major) and 191 -> 152 us (DOF-major).  Element-major direct
// stores (64-byte pieces of each element's run, completed in L2 by other
// row blocks) stay ordinary stores: streaming them doubled the time.
// The hint is applied only to outputs of at least 32 MiB (stream_out, set
// by the host): a launch ends when its writes are acknowledged, and for small
// outputs the streamed writes' longer acknowledgement shows as launch latency
// (512 separate small contractions: 9.1 -> 12.3 ms with the hint everywhere).
__device__ __forceinline__ void store_stream(const ContractArgs& a, float* p, const f4& v) {
    if (a.stream_out)  // uniform
        __builtin_nontemporal_store(v, reinterpret_cast<f4*>(p));
    else
        *reinterpret_cast<f4*>(p) = v;
}

// Write-back of one chunk of a wave's row blocks (p = pc + q*WPE, q < PMAX).
// Element-major: lane l holds stacked rows R0 .. R0+3 (R0 = 16p + 4(l/16))
// of element e; with Np % 4 == 0 they belong to one operator k = R0 / Np.
// DOF-major: lane l holds stacked row R = 16p + l%16 of four elements, and
// out[k][i][.] is row R of out viewed as [K*Np][E].
template <int LAYOUT, int PMAX, int WPE>
__device__ __forceinline__ void store_pairs(const ContractArgs& a, const f4 (&acc)[PMAX], int pc,
                                            int64_t eb0, int lane) {
    const int rows = a.K * a.Np;
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
        const int p = pc + q * WPE;
        if (p >= a.nrb) continue;
        if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
            const int64_t e = eb0 + (lane & 15);
            const int R0 = 16 * p + 4 * (lane >> 4);
            int k = row_op(a, R0), i = R0 - k * a.Np;
            if (e < a.E) {
                if (a.np_vec) {
                    if (R0 < rows)
                        *reinterpret_cast<f4*>(a.out + ((int64_t)k * a.E + e) * a.Np + i) = acc[q];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {  // rows may run into the next operator
                        if (R0 + r < rows) a.out[((int64_t)k * a.E + e) * a.Np + i] = acc[q][r];
                        if (++i == a.Np) i = 0, ++k;
                    }
                }
            }
        } else {
            const int R = 16 * p + (lane & 15);
            const int64_t e = eb0 + 4 * (lane >> 4);
            if (R < rows && e < a.E) {
                float* dst = a.out + (int64_t)R * a.E + e;
                if (a.e_vec) {
                    store_stream(a, dst, acc[q]);
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (e + r < a.E) dst[r] = acc[q][r];
                }
            }
        }
    }
}

// Staged output tile (prefetch bit 3).  Compute waves write their
// accumulators to an LDS slot; store waves copy the slot to `out` with
// contiguous 16-byte stores.
//   element-major: slot float (k*TILE_E + r)*Np + i, so each k's part is
//                  the contiguous run out[k][e0 .. e0+nvalid)[0 .. Np);
//   DOF-major:     slot float (k*Np + i)*(TILE_E + 4) + r (rows padded by
//                  4 floats against LDS bank conflicts); each (k, i) row is
//                  the segment out[k][i][e0 .. e0+nvalid).
template <int LAYOUT, int PMAX, int WPE, int TILE_E>
__device__ __forceinline__ void stage_pairs(const ContractArgs& a, const f4 (&acc)[PMAX], int pc,
                                            int row0, float* os, int lane) {
    const int rows = a.K * a.Np;
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
        const int p = pc + q * WPE;
        if (p >= a.nrb) continue;
        if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
            const int r = row0 + (lane & 15);
            const int R0 = 16 * p + 4 * (lane >> 4);
            int k = row_op(a, R0), i = R0 - k * a.Np;
            if (a.np_vec) {
                if (R0 < rows) *reinterpret_cast<f4*>(os + (k * TILE_E + r) * a.Np + i) = acc[q];
            } else {
#pragma unroll
                for (int r2 = 0; r2 < 4; ++r2) {  // rows may run into the next operator
                    if (R0 + r2 < rows) os[(k * TILE_E + r) * a.Np + i] = acc[q][r2];
                    if (++i == a.Np) i = 0, ++k;
                }
            }
        } else {
            const int R = 16 * p + (lane & 15);
            if (R < rows)
                *reinterpret_cast<f4*>(os + R * (TILE_E + 4) + row0 + 4 * (lane >> 4)) = acc[q];
        }
    }
}

// Store wave sw (of NSW) copies the staged tile at element e0 (nvalid
// valid elements) from slot `os` to `out`.  Store waves issue no global
// loads, so nothing ever waits for their stores.
// 16-byte store, streaming (non-temporal) when NT: the store waves' loops
// are compiled once per kind, so no store carries a branch on stream_out.
template <bool NT>
__device__ __forceinline__ void store_f4(float* p, const f4& v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, reinterpret_cast<f4*>(p));
    else
        *reinterpret_cast<f4*>(p) = v;
}

template <int LAYOUT, int TILE_E, int NSW, bool NT>
__device__ __forceinline__ void store_tile_as(const ContractArgs& a, const float* os, int64_t e0,
                                              int nvalid, int sw, int lane) {
    constexpr int U = 4;  // chunks read from LDS before their stores
    constexpr int STRIDE = 64 * NSW;
    if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
        const int run = nvalid * a.Np;  // floats of one k
        for (int k = 0; k < a.K; ++k) {
            float* g = a.out + ((int64_t)k * a.E + e0) * a.Np;
            const float* src = os + k * TILE_E * a.Np;
            if (a.np_vec) {  // run % 4 == 0; g is 16-byte aligned
                const int nch = run >> 2;
                for (int c0 = 64 * sw + lane; c0 < nch; c0 += STRIDE * U) {
                    f4 v[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int c = c0 + STRIDE * u;
                        v[u] = reinterpret_cast<const f4*>(src)[c < nch ? c : nch - 1];
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int c = c0 + STRIDE * u;
                        if (c < nch) store_f4<NT>(g + 4 * c, v[u]);
                    }
                }
            } else {
                for (int f = 64 * sw + lane; f < run; f += STRIDE) g[f] = src[f];
            }
        }
    } else {
        constexpr int CPR = TILE_E / 4;  // 16-byte chunks per row
        constexpr int LDR = TILE_E + 4;  // padded slot row
        const int rows = a.K * a.Np;
        if (a.e_vec) {  // E % 4 == 0: nvalid % 4 == 0 and every row segment is aligned
            // Chunk c = 64*sw + lane + STRIDE*m is row c / CPR, column 4*(c % CPR):
            // CPR divides 64, so a lane keeps its column and moves RSTEP rows
            // per step (pointers advanced, no per-chunk division).
            constexpr int RSTEP = STRIDE / CPR;
            const int col = 4 * (lane % CPR);
            const bool colok = col < nvalid;
            int row = (64 * sw + lane) / CPR;
            float* dst = a.out + (int64_t)row * a.E + e0 + col;
            const int64_t dstep = (int64_t)RSTEP * a.E;
            for (; row < rows; row += RSTEP * U) {
                f4 v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int rr = row + RSTEP * u < rows ? row + RSTEP * u : rows - 1;
                    v[u] = *reinterpret_cast<const f4*>(os + rr * LDR + col);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (row + RSTEP * u < rows && colok) store_f4<NT>(dst + u * dstep, v[u]);
                }
                dst += U * dstep;
            }
        } else {
            const int n = rows * TILE_E;
            for (int f = 64 * sw + lane; f < n; f += STRIDE) {
                const int row = f / TILE_E, r = f % TILE_E;
                if (r < nvalid) a.out[(int64_t)row * a.E + e0 + r] = os[row * LDR + r];
            }
        }
    }
}

// Copy-out of one staged output tile by the store waves.
template <int LAYOUT, int TILE_E, int NSW>
__device__ __forceinline__ void store_tile(const ContractArgs& a, const float* os, int64_t e0,
                                           int nvalid, int sw, int lane) {
    if (a.stream_out)  // uniform
        store_tile_as<LAYOUT, TILE_E, NSW, true>(a, os, e0, nvalid, sw, lane);
    else
        store_tile_as<LAYOUT, TILE_E, NSW, false>(a, os, e0, nvalid, sw, lane);
}

// dG volume term, write-back of a staged tile: the slot holds the K
// reference derivatives (layout of stage_pairs) and the tile's geometric
// factors at gs (element-major: gs[r*K*K + d*K + k] for element e0 + r;
// DOF-major: gs[(d*K + k)*TILE_E + r]); store wave sw writes
// out[d] = sum_k G(e,d,k) * slot[k] (FP32, k increasing) for d < K.
template <int LAYOUT, int TILE_E, int NSW, bool NT>
__device__ __forceinline__ void store_tile_dg_as(const ContractArgs& a, const float* os,
                                                 const float* gs, int64_t e0, int nvalid, int sw,
                                                 int lane) {
    constexpr int STRIDE = 64 * NSW;
    constexpr int KM = LPX_DG_MAX_K;
    const int K = a.K, KK = a.K * a.K;
    if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
        const int run = nvalid * a.Np;  // floats of one d
        if (a.np_vec) {
            // A chunk (4 floats of one element) is read once for all K outputs:
            // the K reference derivatives and the element's K x K factors.
            // U chunks are read before any is combined and stored.
            constexpr int U = 2;
            const int nch = run >> 2;
            for (int c0 = 64 * sw + lane; c0 < nch; c0 += STRIDE * U) {
                f4 v[U][KM];
                float gk[U][KM][KM];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    int c = c0 + STRIDE * u;
                    c = c < nch ? c : nch - 1;
                    const int r = row_op(a, 4 * c), i = 4 * c - r * a.Np;
#pragma unroll
                    for (int k = 0; k < KM; ++k) {
                        if (k < K) {
                            v[u][k] = *reinterpret_cast<const f4*>(os + (k * TILE_E + r) * a.Np + i);
#pragma unroll
                            for (int d = 0; d < KM; ++d)
                                if (d < K) gk[u][d][k] = gs[r * KK + d * K + k];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = c0 + STRIDE * u;
                    if (c >= nch) continue;
#pragma unroll
                    for (int d = 0; d < KM; ++d) {
                        if (d >= K) continue;
                        f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                        for (int k = 0; k < KM; ++k)
                            if (k < K) {
#pragma unroll
                                for (int t = 0; t < 4; ++t)
                                    acc[t] = fmaf(gk[u][d][k], v[u][k][t], acc[t]);
                            }
                        store_f4<NT>(a.out + ((int64_t)d * a.E + e0) * a.Np + 4 * c, acc);
                    }
                }
            }
        } else {
            for (int d = 0; d < K; ++d) {
                float* g = a.out + ((int64_t)d * a.E + e0) * a.Np;
                for (int f = 64 * sw + lane; f < run; f += STRIDE) {
                    const int r = row_op(a, f);
                    const int i = f - r * a.Np;
                    float acc = 0.0f;
#pragma unroll
                    for (int k = 0; k < KM; ++k)
                        if (k < K) acc = fmaf(gs[r * KK + d * K + k], os[(k * TILE_E + r) * a.Np + i], acc);
                    g[f] = acc;
                }
            }
        }
    } else {
        constexpr int CPR = TILE_E / 4;  // 16-byte chunks per row
        constexpr int LDR = TILE_E + 4;  // padded slot row
        if (a.e_vec) {
            // A lane keeps one column chunk and walks rows i of the operator:
            // its factors (K*K chunks of the G area) are read once per tile,
            // the K slot rows k*Np + i once per row for all K outputs.
            constexpr int RSTEP = STRIDE / CPR;
            const int col = 4 * (lane % CPR);
            const bool colok = col < nvalid;
            f4 gk[KM][KM];
#pragma unroll
            for (int d = 0; d < KM; ++d)
#pragma unroll
                for (int k = 0; k < KM; ++k)
                    if (d < K && k < K)
                        gk[d][k] = *reinterpret_cast<const f4*>(gs + (d * K + k) * TILE_E + col);
            for (int i = (64 * sw + lane) / CPR; i < a.Np; i += RSTEP) {
                f4 v[KM];
#pragma unroll
                for (int k = 0; k < KM; ++k)
                    if (k < K) v[k] = *reinterpret_cast<const f4*>(os + (k * a.Np + i) * LDR + col);
#pragma unroll
                for (int d = 0; d < KM; ++d) {
                    if (d >= K) continue;
                    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int k = 0; k < KM; ++k)
                        if (k < K) {
#pragma unroll
                            for (int t = 0; t < 4; ++t) acc[t] = fmaf(gk[d][k][t], v[k][t], acc[t]);
                        }
                    if (colok)
                        store_f4<NT>(a.out + (int64_t)(d * a.Np + i) * a.E + e0 + col, acc);
                }
            }
        } else {
            const int n = K * a.Np * TILE_E;
            for (int f = 64 * sw + lane; f < n; f += STRIDE) {
                const int row = f / TILE_E, r = f % TILE_E;
                if (r >= nvalid) continue;
                const int d = row_op(a, row), i = row - d * a.Np;
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < KM; ++k)
                    if (k < K)
                        acc = fmaf(gs[(d * K + k) * TILE_E + r], os[(k * a.Np + i) * LDR + r], acc);
                a.out[(int64_t)row * a.E + e0 + r] = acc;
            }
        }
    }
}

template <int LAYOUT, int TILE_E, int NSW>
__device__ __forceinline__ void store_tile_dg(const ContractArgs& a, const float* os,
                                              const float* gs, int64_t e0, int nvalid, int sw,
                                              int lane) {
    if (a.stream_out)  // uniform
        store_tile_dg_as<LAYOUT, TILE_E, NSW, true>(a, os, gs, e0, nvalid, sw, lane);
    else
        store_tile_dg_as<LAYOUT, TILE_E, NSW, false>(a, os, gs, e0, nvalid, sw, lane);
}

// dG volume term: the compute waves copy a tile's geometric factors into its
// staged output slot (they issue no other global access in the staged-output
// pipeline when D sits in LDS or registers, so waiting for these loads costs
// nothing else).  Compute wave cw (of NCW) loads floats f = cw*64 + lane +
// 64*NCW*q of the tile's factors: element-major the run G[e0*K*K ..), DOF-
// major row f / TILE_E (= d*K + k) at element f % TILE_E.  Reads past the
// tile are clamped in bounds and never stored past the slot's G area.
template <int TILE_E, int NCW>
struct GTile {
    static constexpr int Q = (TILE_E * LPX_DG_MAX_K * LPX_DG_MAX_K + 64 * NCW - 1) / (64 * NCW);
};

template <int LAYOUT, int TILE_E, int NCW>
__device__ __forceinline__ void g_tile_load(const ContractArgs& a, int64_t e0, int nvalid, int cw,
                                            int lane, float (&gv)[GTile<TILE_E, NCW>::Q]) {
    const int KK = a.K * a.K;
#pragma unroll
    for (int q = 0; q < GTile<TILE_E, NCW>::Q; ++q) {
        const int f = cw * 64 + lane + 64 * NCW * q;
        if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
            const int nflat = nvalid * KK;
            gv[q] = a.G[e0 * KK + (f < nflat ? f : nflat - 1)];
        } else {
            const int row = f / TILE_E, r = f % TILE_E;
            gv[q] = a.G[(int64_t)(row < KK ? row : KK - 1) * a.E + e0 + (r < nvalid ? r : nvalid - 1)];
        }
    }
}

template <int TILE_E, int NCW>
__device__ __forceinline__ void g_tile_store(const ContractArgs& a, float* gs, int cw, int lane,
                                             const float (&gv)[GTile<TILE_E, NCW>::Q]) {
    const int n = TILE_E * a.K * a.K;
#pragma unroll
    for (int q = 0; q < GTile<TILE_E, NCW>::Q; ++q) {
        const int f = cw * 64 + lane + 64 * NCW * q;
        if (f < n) gs[f] = gv[q];
    }
}

// One wave's share of a 16-element block starting at element eb0: the
// (k, i-block) pairs p = part, part + WPE, ... (WPE waves share a block);
// for each, the MFMA chain over the k-steps of j, then the write-back.
// D fragments come from LDS (PF_D) or global memory; u fragments from the
// staged tile `ut` at row `row0` (PF_U) or global memory.  The summation
// order of every output depends only on PREC: all records of a precision
// give bit-identical results.
// MASK (fp32): zero u columns j >= Np.  It is needed only when Np % 4 != 0:
// otherwise the quads and the steps after them cover exactly j < Np, and
// dropping the selects keeps their lane masks out of the scalar registers.
// bf16/bf16x3 mask their last k-step only (it straddles Np unless
// Np % 32 == 0); the other steps lie below Np.
// Row blocks a wave holds per chunk: a three-operator block's share, at
// most 6 (larger shares run in several chunks, re-reading u).
template <int NTMAX, int WPE>
constexpr int pmax_cap() {
    return (3 * NTMAX + WPE - 1) / WPE < 6 ? (3 * NTMAX + WPE - 1) / WPE : 6;
}

// Calls f(std::integral_constant<int, P>()) with P row blocks per wave and
// chunk, P <= CAP, enough to cover all nrb row blocks in one chunk when CAP
// is: a problem with fewer operators or rows than the kernel is built for
// then runs fewer MFMA chains on duplicate blocks.  MODE 0 builds P = CAP
// only; MODE 1 adds one smaller size (1 of 2, 2 of 3, 4 of 6); MODE 2
// builds every P in 1..CAP (for one kernel serving many shapes).  The modes
// bound the code built per kernel.  nrb is uniform, so is the branch.
template <int CAP, int WPE, int MODE, class F>
__device__ __forceinline__ void with_pmax(int nrb, F&& f) {
    const int need = (nrb + WPE - 1) / WPE;
    if constexpr (MODE == 2) {
        if constexpr (CAP > 1) if (need <= 1) return f(std::integral_constant<int, 1>());
        if constexpr (CAP > 2) if (need <= 2) return f(std::integral_constant<int, 2>());
        if constexpr (CAP > 3) if (need <= 3) return f(std::integral_constant<int, 3>());
        if constexpr (CAP > 4) if (need <= 4) return f(std::integral_constant<int, 4>());
        if constexpr (CAP > 5) if (need <= 5) return f(std::integral_constant<int, 5>());
    } else if constexpr (MODE == 1) {
        constexpr int SMALL = CAP == 6 ? 4 : CAP - 1;
        if constexpr (SMALL >= 1) if (need <= SMALL) return f(std::integral_constant<int, SMALL>());
    }
    f(std::integral_constant<int, CAP>());
}

// FP32 MFMAs cost about five times the bf16x3 triple per output, so only
// the FP32 kernels past 32 rows are built with a smaller row-block size.
template <int PREC, int NTMAX>
constexpr int pmax_mode() {
    return PREC == LPX_FP32 && NTMAX >= 4 ? 1 : 0;
}

template <int PREC, int LAYOUT, int NTMAX, bool PF_D, bool PF_U, int TILE_E, int WPE, int UNROLL,
          bool PF_O = false, bool MASK = true, int PM = pmax_cap<NTMAX, WPE>(),
          bool DGLOBAL = false>
__device__ __forceinline__ void block_compute(const ContractArgs& a, const unsigned char* lds,
                                              const float* ut, int row0, int64_t eb0, int part,
                                              int lane, float* os = nullptr) {
    constexpr int PMAX = PM;
    const int npairs = a.nrb;
    const int64_t nfrag = (int64_t)npairs * a.nsteps * 64;
    for (int pc = part; pc < npairs; pc += WPE * PMAX) {
        f4 acc[PMAX];
        int pp[PMAX];
#pragma unroll
        for (int q = 0; q < PMAX; ++q) {
            acc[q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            const int p = pc + q * WPE;
            pp[q] = p < npairs ? p : npairs - 1;  // clamped: a duplicate block is loaded, never used
        }
        auto step = [&](int s, auto masked) {
            Frag<PREC> uf;
            if constexpr (PF_U)
                uf = u_frag_lds<PREC, LAYOUT, TILE_E, decltype(masked)::value>(
                    ut, a.Np, a.np_vec, row0, s, a.nsteps & ~3, lane);
            else
                uf = u_frag_global<PREC, LAYOUT>(a, eb0, s, lane);
            // every held pair runs: a pair past the last one holds a clamped
            // duplicate and is never stored (no branch between the MFMAs)
#pragma unroll
            for (int q = 0; q < PMAX; ++q) {
                Frag<PREC> df;
                if constexpr (PF_D)
                    df = d_frag_lds<PREC, DGLOBAL>(lds, nfrag, (pp[q] * a.nsteps + s) * 64 + lane);
                else
                    df = d_frag_global<PREC>(a, pp[q], s, lane);
                if constexpr (LAYOUT == LPX_ELEMENT_MAJOR)
                    acc[q] = mma(df, uf, acc[q]);  // rows i, columns e
                else
                    acc[q] = mma(uf, df, acc[q]);  // rows e, columns i
            }
        };
        int s = 0;
        if constexpr (PREC == LPX_FP32) {
            // Whole quads: one 16-byte read per operand, then four MFMAs
            // per pair; UNROLL counts quads.
            auto quad = [&](int Q) {
                f4 uq;
                if constexpr (PF_U)
                    uq = u_quad_lds<LAYOUT, TILE_E, MASK>(ut, a.Np, a.np_vec, row0, Q, lane);
                else
                    uq = u_quad_global<LAYOUT>(a, eb0, Q, lane);
                f4 dq[PMAX];
#pragma unroll
                for (int q = 0; q < PMAX; ++q) {
                    if constexpr (PF_D)
                        dq[q] = d_quad_lds<DGLOBAL>(lds, pp[q], Q, a.nsteps, lane);
                    else
                        dq[q] = d_quad_global(a, pp[q], Q, lane);
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) {
#pragma unroll
                    for (int q = 0; q < PMAX; ++q) {
                        const Frag<PREC> df{dq[q][m]}, uf{uq[m]};
                        if constexpr (LAYOUT == LPX_ELEMENT_MAJOR)
                            acc[q] = mma(df, uf, acc[q]);
                        else
                            acc[q] = mma(uf, df, acc[q]);
                    }
                }
            };
            const int nq = a.nsteps >> 2;
            int Q = 0;
            for (; Q + UNROLL <= nq; Q += UNROLL) {
#pragma unroll
                for (int uu = 0; uu < UNROLL; ++uu) quad(Q + uu);
            }
            for (; Q < nq; ++Q) quad(Q);
            for (s = 4 * nq; s < a.nsteps; ++s) step(s, std::integral_constant<bool, MASK>());
        } else {
            const int last = a.nsteps - 1;  // the only step that can straddle Np
            for (; s + UNROLL <= last; s += UNROLL) {
#pragma unroll
                for (int uu = 0; uu < UNROLL; ++uu) step(s + uu, std::false_type());
            }
            for (; s < last; ++s) step(s, std::false_type());
            step(last, std::true_type());
        }
        if constexpr (PF_O)
            stage_pairs<LAYOUT, PMAX, WPE, TILE_E>(a, acc, pc, row0, os, lane);
        else
            store_pairs<LAYOUT, PMAX, WPE>(a, acc, pc, eb0, lane);
    }
}

// D held in registers (precompute into private memory, sec. 2.4.4): each
// wave loads the D fragments of its own pairs once and keeps them for the
// whole kernel.  NS k-steps cover the 16*NTMAX columns; steps past nsteps
// hold zeros.  Needs all of the block's pairs in one chunk: K*nt <= WPE*PMAX.
template <int PREC, int NTMAX, int WPE>
struct DRegs {
    static constexpr int PMAX = (3 * NTMAX + WPE - 1) / WPE;
    static constexpr int NS = 16 * NTMAX / Traits<PREC>::KSTEP;
    static constexpr int NT = PREC == LPX_FP32 ? 3 : 1;  // fp32 steps after the last quad
    Frag<PREC> f[PMAX][NS];
    Frag<PREC> t[PMAX][NT];  // fp32: step 4*(nsteps/4) + m, so its register is fixed
};

template <int PREC, int NTMAX, int WPE>
__device__ __forceinline__ void load_dregs(const ContractArgs& a, int part, int lane,
                                           DRegs<PREC, NTMAX, WPE>& d) {
    using DR = DRegs<PREC, NTMAX, WPE>;
#pragma unroll
    for (int q = 0; q < DR::PMAX; ++q) {
        int p = part + q * WPE;
        p = p < a.nrb ? p : a.nrb - 1;  // clamped: the duplicate is never used
#pragma unroll
        for (int s = 0; s < DR::NS; ++s) d.f[q][s] = d_frag_global<PREC>(a, p, s, lane);
        if constexpr (PREC == LPX_FP32) {
#pragma unroll
            for (int m = 0; m < DR::NT; ++m)
                d.t[q][m] = d_frag_global<PREC>(a, p, (a.nsteps & ~3) + m, lane);
        }
    }
}

// u operands of one 16-element block for the register-D routine: fp32 quads
// and the steps after the last quad, or bf16 steps.
template <int PREC, int NTMAX, int WPE>
struct UOps {
    using DR = DRegs<PREC, NTMAX, WPE>;
    static constexpr int NQ = PREC == LPX_FP32 ? DR::NS / 4 : 1;
    static constexpr int NSB = PREC == LPX_FP32 ? 1 : DR::NS;
    f4 uq[NQ];
    Frag<PREC> ut3[DR::NT];
    Frag<PREC> uf[NSB];
};

// Every u operand of a block is read at once, without branches (reads past
// the last step are in bounds and, where they can reach j >= Np, masked),
// so the reads overlap one another and the wave waits once.
template <int PREC, int LAYOUT, int NTMAX, bool PF_U, int TILE_E, int WPE, bool MASK>
__device__ __forceinline__ UOps<PREC, NTMAX, WPE> dreg_read(const ContractArgs& a, const float* ut,
                                                            int row0, int64_t eb0, int lane) {
    using DR = DRegs<PREC, NTMAX, WPE>;
    UOps<PREC, NTMAX, WPE> o;
    if constexpr (PREC == LPX_FP32) {
        const int nq = a.nsteps >> 2;
#pragma unroll
        for (int Q = 0; Q < o.NQ; ++Q) {
            if constexpr (PF_U)
                o.uq[Q] = u_quad_lds<LAYOUT, TILE_E, MASK>(ut, a.Np, a.np_vec, row0, Q, lane);
            else
                o.uq[Q] = u_quad_global<LAYOUT>(a, eb0, Q, lane);
        }
#pragma unroll
        for (int m = 0; m < DR::NT; ++m) {
            if constexpr (PF_U)
                o.ut3[m] = u_frag_lds<PREC, LAYOUT, TILE_E, MASK>(ut, a.Np, a.np_vec, row0,
                                                                  4 * nq + m, 4 * nq, lane);
            else
                o.ut3[m] = u_frag_global<PREC, LAYOUT>(a, eb0, 4 * nq + m, lane);
        }
    } else {
#pragma unroll
        for (int s = 0; s < DR::NS; ++s) {
            // nsteps == NS for every Np of the NTMAX bucket, so only the last
            // compiled step straddles Np
            if constexpr (PF_U) {
                if (s == DR::NS - 1)
                    o.uf[s] = u_frag_lds<PREC, LAYOUT, TILE_E, true>(ut, a.Np, a.np_vec, row0, s,
                                                                     0, lane);
                else
                    o.uf[s] = u_frag_lds<PREC, LAYOUT, TILE_E, false>(ut, a.Np, a.np_vec, row0,
                                                                      s, 0, lane);
            } else {
                o.uf[s] = u_frag_global<PREC, LAYOUT>(a, eb0, s, lane);
            }
        }
    }
    return o;
}

// The MFMA chains of one block from its u operands, then the write-back.
// MFMAs run for every held pair (a pair past the last one holds a
// duplicate and is never stored), so the only branches are one per k-step
// group, with constant register indices throughout.
template <int PREC, int LAYOUT, int NTMAX, int TILE_E, int WPE, bool PF_O>
__device__ __forceinline__ void dreg_mma_store(const ContractArgs& a,
                                               const DRegs<PREC, NTMAX, WPE>& d,
                                               const UOps<PREC, NTMAX, WPE>& o, int row0,
                                               int64_t eb0, int part, int lane, float* os) {
    using DR = DRegs<PREC, NTMAX, WPE>;
    f4 acc[DR::PMAX];
#pragma unroll
    for (int q = 0; q < DR::PMAX; ++q) acc[q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    auto mma_all = [&](const Frag<PREC> (&df)[DR::PMAX], const Frag<PREC>& uf) {
#pragma unroll
        for (int q = 0; q < DR::PMAX; ++q) {
            if constexpr (LAYOUT == LPX_ELEMENT_MAJOR)
                acc[q] = mma(df[q], uf, acc[q]);
            else
                acc[q] = mma(uf, df[q], acc[q]);
        }
    };
    if constexpr (PREC == LPX_FP32) {
        const int nq = a.nsteps >> 2;
        const int ntail = a.nsteps - 4 * nq;  // 0..3 steps after the last quad
#pragma unroll
        for (int Q = 0; Q < o.NQ; ++Q) {
            if (Q < nq) {
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    Frag<PREC> df[DR::PMAX];
#pragma unroll
                    for (int q = 0; q < DR::PMAX; ++q) df[q] = d.f[q][4 * Q + m];
                    mma_all(df, Frag<PREC>{o.uq[Q][m]});
                }
            }
        }
#pragma unroll
        for (int m = 0; m < DR::NT; ++m) {
            if (m < ntail) {
                Frag<PREC> df[DR::PMAX];
#pragma unroll
                for (int q = 0; q < DR::PMAX; ++q) df[q] = d.t[q][m];
                mma_all(df, o.ut3[m]);
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < DR::NS; ++s) {
            if (s < a.nsteps) {
                Frag<PREC> df[DR::PMAX];
#pragma unroll
                for (int q = 0; q < DR::PMAX; ++q) df[q] = d.f[q][s];
                mma_all(df, o.uf[s]);
            }
        }
    }
    if constexpr (PF_O)
        stage_pairs<LAYOUT, DR::PMAX, WPE, TILE_E>(a, acc, part, row0, os, lane);
    else
        store_pairs<LAYOUT, DR::PMAX, WPE>(a, acc, part, eb0, lane);
}

template <int PREC, int LAYOUT, int NTMAX, bool PF_U, int TILE_E, int WPE, bool PF_O = false,
          bool MASK = true>
__device__ __forceinline__ void block_compute_dreg(const ContractArgs& a,
                                                   const DRegs<PREC, NTMAX, WPE>& d,
                                                   const float* ut, int row0, int64_t eb0,
                                                   int part, int lane, float* os = nullptr) {
    const auto o = dreg_read<PREC, LAYOUT, NTMAX, PF_U, TILE_E, WPE, MASK>(a, ut, row0, eb0, lane);
    dreg_mma_store<PREC, LAYOUT, NTMAX, TILE_E, WPE, PF_O>(a, d, o, row0, eb0, part, lane, os);
}

// ------------------------------------------------------------ the kernel
// Work-group shape (contract_shape).  Without a staged u tile: four waves
// per 16-element block, splitting its (k, i-block) pairs.  With one:
// NCW = min(4 * TILE_E/16, 8) compute waves (WPE per block), NLW loader
// waves and, with a staged output tile, NSW store waves.
template <int TILE_E, int NTMAX, int PREFETCH>
struct Shape {
    static constexpr ContractShape CS = contract_shape(TILE_E, NTMAX, PREFETCH);
    static constexpr int NCW = CS.ncw, WPE = CS.wpe, BPW = CS.bpw, NLW = CS.nlw,
                         NSW = CS.nsw, THREADS = CS.threads;
};

// The work of one work-group on tiles t0 + n * g, n < nmine, of the
// contraction `a`: the whole kernel (contract_kernel) or one run of a
// batch (contract_runs_kernel).
// EPI = 1: the dG volume term (needs PREFETCH bit 3): the tile's geometric
// factors travel with its staged output and the store waves apply them.
template <int PREC, int LAYOUT, int NTMAX, int TILE_E, int PREFETCH, int UNROLL, int EPI>
__device__ __forceinline__ void contract_tiles(const ContractArgs& a, int64_t t0, int64_t g,
                                               int64_t nmine, int tid) {
    static_assert(EPI == 0 || (PREFETCH & 8), "the dG epilogue runs in the store waves");
    extern __shared__ __align__(16) unsigned char lds[];
    using S = Shape<TILE_E, NTMAX, PREFETCH>;
    constexpr bool PF_D = (PREFETCH & 1) != 0;
    constexpr bool PF_U = (PREFETCH & 2) != 0;
    constexpr bool D_REG = (PREFETCH & 4) != 0;
    constexpr bool PF_O = (PREFETCH & 8) != 0;

    const int lane = tid & 63;
    // the same in every lane of a wave: scalar, so role branches and
    // per-wave LDS addresses stay in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t nfrag = (int64_t)a.nrb * a.nsteps * 64;
    float* ring = reinterpret_cast<float*>(
        lds + (PF_D ? nfrag * Lds<PREC>::DFRAG_BYTES * Lds<PREC>::PLANES : 0));
    float* oring = ring + 4 * a.ldu;  // staged output slots follow the u slots

    if constexpr (PF_D) stage_d<PREC, S::THREADS>(a, lds, tid);
    // With a staged u tile every role has written part of D: one full
    // barrier (LDS writes complete, then s_barrier) before any role goes on,
    // since the loader waves' own barriers do not wait for LDS writes.
    if constexpr (PF_D && PF_U) __syncthreads();

    if constexpr (!PF_U) {
        if constexpr (PF_D) __syncthreads();
        const int eblk = wave / S::WPE, part = wave % S::WPE;
        if constexpr (D_REG) {
            DRegs<PREC, NTMAX, S::WPE> d;
            load_dregs<PREC, NTMAX, S::WPE>(a, part, lane, d);
            for (int64_t n = 0; n < nmine; ++n) {
                const int64_t e0 = (t0 + n * g) * TILE_E;
                if (e0 + 16 * eblk >= a.E) continue;
                block_compute_dreg<PREC, LAYOUT, NTMAX, false, TILE_E, S::WPE>(
                    a, d, nullptr, 0, e0 + 16 * eblk, part, lane);
            }
        } else {
            with_pmax<pmax_cap<NTMAX, S::WPE>(), S::WPE, pmax_mode<PREC, NTMAX>()>(a.nrb, [&](auto pm) {
                for (int64_t n = 0; n < nmine; ++n) {
                    const int64_t e0 = (t0 + n * g) * TILE_E;
                    if (e0 + 16 * eblk >= a.E) continue;  // uniform per wave; no barrier below
                    // D from LDS, or from its arrangement in global memory
                    block_compute<PREC, LAYOUT, NTMAX, true, false, TILE_E, S::WPE, UNROLL, false,
                                  true, decltype(pm)::value, !PF_D>(
                        a, PF_D ? lds : a.Darr, nullptr, 0, e0 + 16 * eblk, part, lane);
                }
            });
        }
    } else {
        // The work-group's n-th tile is t0 + n * g, n < nmine.
        // Every wave runs `niter` iterations of one barrier each (one more
        // than nmine when store waves trail the compute waves by a tile):
        //   iteration n: loaders start tile n+3 into u slot (n+3)&3 and wait
        //   for tile n+1; compute waves work on tile n from u slot n&3
        //   (writing output slot n&1 when staged); store waves copy output
        //   slot (n-1)&1 to global memory.
        // Each slot is rewritten only in an iteration after the one that
        // read it, so the barrier ending each iteration orders every access.
        const int64_t niter = PF_O ? nmine + 1 : nmine;
        auto nvalid_of = [&](int64_t tile) {
            const int64_t rest = a.E - tile * TILE_E;
            return (int)(rest < TILE_E ? rest : TILE_E);
        };
        if (wave >= S::NCW + S::NLW) {
            if constexpr (PF_O) {
                const int sw = wave - S::NCW - S::NLW;
                __syncthreads();
                for (int64_t n = 0; n < niter; ++n) {
                    if (n >= 1) {
                        const int64_t tile = t0 + (n - 1) * g;
                        const float* os = oring + ((n - 1) & 1) * a.ldo;
                        if constexpr (EPI)
                            store_tile_dg<LAYOUT, TILE_E, S::NSW>(a, os, os + a.ldo_g,
                                                                  tile * TILE_E, nvalid_of(tile),
                                                                  sw, lane);
                        else
                            store_tile<LAYOUT, TILE_E, S::NSW>(a, os, tile * TILE_E,
                                                               nvalid_of(tile), sw, lane);
                    }
                    __syncthreads();
                }
            }
        } else if (wave >= S::NCW) {
            const int lw = wave - S::NCW;
            loader_loop<Loader<TILE_E, NTMAX, S::NLW>::PER_LANE>(nmine, niter, [&](int64_t n) {
                const int64_t tile = t0 + n * g;
                return loader_issue<LAYOUT, TILE_E, NTMAX, S::NLW>(
                    a, ring + (n & 3) * a.ldu, tile * TILE_E, nvalid_of(tile), lw, lane);
            });
        } else {
            // Compute wave: part `part` of blocks eblk0, eblk0 + NCW/WPE, ...
            // (BPW blocks of each tile).
            const int eblk0 = wave / S::WPE, part = wave % S::WPE;
            constexpr int BSTRIDE = S::NCW / S::WPE;
            auto tile_work = [&](auto&& block, int64_t n) {
                const int64_t tile = t0 + n * g;
                const int nv = nvalid_of(tile);
                if (nv == TILE_E) {  // uniform: whole tile, no per-block test
#pragma unroll
                    for (int b = 0; b < S::BPW; ++b) block(tile, n, 16 * (eblk0 + b * BSTRIDE));
                } else {
#pragma unroll
                    for (int b = 0; b < S::BPW; ++b)
                        if (16 * (eblk0 + b * BSTRIDE) < nv)
                            block(tile, n, 16 * (eblk0 + b * BSTRIDE));
                }
            };
            // dG volume term: the tile's geometric factors are loaded before
            // its MFMA work and written to its output slot after it
            auto with_g = [&](int64_t n, auto&& work) {
                if constexpr (EPI) {
                    const int64_t tile = t0 + n * g;
                    float gv[GTile<TILE_E, S::NCW>::Q];
                    g_tile_load<LAYOUT, TILE_E, S::NCW>(a, tile * TILE_E, nvalid_of(tile), wave,
                                                        lane, gv);
                    work();
                    g_tile_store<TILE_E, S::NCW>(a, oring + (n & 1) * a.ldo + a.ldo_g, wave,
                                                 lane, gv);
                } else {
                    work();
                }
            };
            if constexpr (D_REG) {
                DRegs<PREC, NTMAX, S::WPE> d;
                load_dregs<PREC, NTMAX, S::WPE>(a, part, lane, d);
                auto block = [&](int64_t tile, int64_t n, int row0) {
                    auto run = [&](auto mask) {
                        block_compute_dreg<PREC, LAYOUT, NTMAX, true, TILE_E, S::WPE, PF_O,
                                           decltype(mask)::value>(
                            a, d, ring + (n & 3) * a.ldu, row0, tile * TILE_E + row0, part, lane,
                            oring + (n & 1) * a.ldo);
                    };
                    if (PREC == LPX_FP32 && a.np_vec)  // uniform
                        run(std::false_type());
                    else
                        run(std::true_type());
                };
                // Four blocks per tile (one compute wave per SIMD): block b+1's
                // operands are read before block b's MFMAs, so the wave's own
                // MFMAs hide its LDS latency.
                auto pipelined = [&](int64_t n) {
                    const int64_t tile = t0 + n * g;
                    const int nv = nvalid_of(tile);
                    auto run = [&](auto mask) {
                        constexpr bool M = decltype(mask)::value;
                        const float* ut = ring + (n & 3) * a.ldu;
                        float* os = oring + (n & 1) * a.ldo;
                        auto row = [&](int b) { return 16 * (eblk0 + b * BSTRIDE); };
                        auto o = dreg_read<PREC, LAYOUT, NTMAX, true, TILE_E, S::WPE, M>(
                            a, ut, row(0), tile * TILE_E + row(0), lane);
#pragma unroll
                        for (int b = 0; b < S::BPW; ++b) {
                            const auto cur = o;
                            if (b + 1 < S::BPW)
                                o = dreg_read<PREC, LAYOUT, NTMAX, true, TILE_E, S::WPE, M>(
                                    a, ut, row(b + 1), tile * TILE_E + row(b + 1), lane);
                            if (row(b) < nv)
                                dreg_mma_store<PREC, LAYOUT, NTMAX, TILE_E, S::WPE, PF_O>(
                                    a, d, cur, row(b), tile * TILE_E + row(b), part, lane, os);
                        }
                    };
                    if (PREC == LPX_FP32 && a.np_vec)  // uniform
                        run(std::false_type());
                    else
                        run(std::true_type());
                };
                __syncthreads();
                for (int64_t n = 0; n < niter; ++n) {
                    if (n < nmine) {
                        with_g(n, [&] {
                            if constexpr (S::BPW == 4)
                                pipelined(n);
                            else
                                tile_work(block, n);
                        });
                    }
                    __syncthreads();
                }
            } else {
                // every compute wave takes the same branch of with_pmax, so
                // the barrier count is that of the other roles
                with_pmax<pmax_cap<NTMAX, S::WPE>(), S::WPE, pmax_mode<PREC, NTMAX>()>(a.nrb, [&](auto pm) {
                    auto block = [&](int64_t tile, int64_t n, int row0) {
                        auto run = [&](auto mask) {
                            // D from LDS, or from its arrangement in global memory
                            block_compute<PREC, LAYOUT, NTMAX, true, true, TILE_E, S::WPE, UNROLL,
                                          PF_O, decltype(mask)::value, decltype(pm)::value, !PF_D>(
                                a, PF_D ? lds : a.Darr, ring + (n & 3) * a.ldu, row0,
                                tile * TILE_E + row0, part, lane, oring + (n & 1) * a.ldo);
                        };
                        if (PREC == LPX_FP32 && a.np_vec)  // uniform
                            run(std::false_type());
                        else
                            run(std::true_type());
                    };
                    __syncthreads();
                    for (int64_t n = 0; n < niter; ++n) {
                        if (n < nmine) with_g(n, [&] { tile_work(block, n); });
                        __syncthreads();
                    }
                });
            }
        }
    }
}

// The arguments of one contraction read from a table in the constant
// address space, field by field (a class object in another address space
// cannot be copied whole): scalar loads, and the pointers read are taken
// to point to global memory.
template <class CItem>
__device__ __forceinline__ ContractArgs load_args(const CItem* p) {
    static_assert(sizeof(ContractArgs) == 120, "load_args copies every field");
    ContractArgs a;
    a.D = p->D;
    a.u = p->u;
    a.out = p->out;
    a.Darr = p->Darr;
    a.E = p->E;
    a.ntiles = p->ntiles;
    a.K = p->K;
    a.Np = p->Np;
    a.nt = p->nt;
    a.nsteps = p->nsteps;
    a.ldu = p->ldu;
    a.nrb = p->nrb;
    a.np_div.m = p->np_div.m;
    a.np_div.sh = p->np_div.sh;
    a.ldo = p->ldo;
    a.G = p->G;
    a.ldo_g = p->ldo_g;
    a.np_vec = p->np_vec;
    a.e_vec = p->e_vec;
    a.stream_out = p->stream_out;
    a.blocked = p->blocked;
    return a;
}

// A 64-bit value known to be the same in every lane, as a scalar.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One contraction over the persistent grid of G work-groups: work-group b
// takes tiles b, b + G, b + 2G, ... (cyclic order), or the consecutive
// tiles b*c .. b*c + c - 1, c = ceil(ntiles / G) (blocked order).
template <int PREC, int LAYOUT, int NTMAX, int TILE_E, int PREFETCH, int UNROLL, int EPI = 0>
__global__ __launch_bounds__((Shape<TILE_E, NTMAX, PREFETCH>::THREADS)) void contract_kernel(
    ContractArgs a) {
    const int64_t b = blockIdx.x, G = gridDim.x;
    int64_t t0 = b, step = G, nmine = b < a.ntiles ? (a.ntiles - 1 - b) / G + 1 : 0;
    if (a.blocked) {  // uniform
        const int64_t c = (a.ntiles + G - 1) / G, rest = a.ntiles - b * c;
        t0 = b * c;
        step = 1;
        nmine = rest < 0 ? 0 : (rest < c ? rest : c);
    }
    // The three values are the same in every lane; without the explicit
    // broadcast the compiler keeps the selected values in vector registers,
    // which made the element-major register-D kernels spill (bf16x3 tile 32:
    // 108 -> 128 VGPRs and 76 bytes of scratch per lane).
    t0 = uniform64(t0);
    step = uniform64(step);
    nmine = uniform64(nmine);
    contract_tiles<PREC, LAYOUT, NTMAX, TILE_E, PREFETCH, UNROLL, EPI>(a, t0, step, nmine,
                                                                       threadIdx.x);
}

// A ragged batch: runs of consecutive tiles of one instance each, listed
// per work-group (runs wg_first[b] .. wg_first[b + 1] - 1 for work-group b).
struct Run {
    int64_t first;  // first tile of the run
    int32_t inst;   // index into `items`
    int32_t count;  // tiles in the run
};
struct RunArgs {
    const ContractArgs* __restrict__ items;
    const Run* __restrict__ runs;
    const int32_t* __restrict__ wg_first;
};

// Every instance of a launch runs the same record's code as a separate
// contraction (its D staged or loaded again at the start of each run), so
// its outputs are those of lpx_contract with that record.
template <int PREC, int LAYOUT, int NTMAX, int TILE_E, int PREFETCH, int UNROLL>
__global__ __launch_bounds__((Shape<TILE_E, NTMAX, PREFETCH>::THREADS)) void contract_runs_kernel(
    RunArgs r) {
    // The tables are read through constant-address-space pointers: they do
    // not change during the launch, so the compiler loads them with scalar
    // loads into scalar registers, and it takes the pointers read from the
    // descriptors to point to global memory (global loads and stores; as
    // generic pointers they gave flat accesses, which also count against the
    // LDS wait counter, and vector copies of every argument).
    typedef __attribute__((address_space(4))) const ContractArgs CItem;
    typedef __attribute__((address_space(4))) const Run CRun;
    typedef __attribute__((address_space(4))) const int32_t CInt;
    const CItem* items = (const CItem*)r.items;
    const CRun* runs = (const CRun*)r.runs;
    const CInt* wg_first = (const CInt*)r.wg_first;
    const int q0 = wg_first[blockIdx.x], q1 = wg_first[blockIdx.x + 1];
    for (int q = q0; q < q1; ++q) {
        // every wave is past its last LDS access of the previous run
        if (q > q0) __syncthreads();
        const int64_t first = runs[q].first;
        const int32_t inst = runs[q].inst, count = runs[q].count;
        const ContractArgs a = load_args(items + inst);
        // The thread index passes through an empty asm statement, so nothing
        // derived from it is computed once before the loop and kept live
        // across every run (that raised the staged kernels to the VGPR cap).
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        contract_tiles<PREC, LAYOUT, NTMAX, TILE_E, PREFETCH, UNROLL, 0>(a, first, 1, count, tid);
    }
}

}  // namespace kern
}  // namespace lpx
