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
//             of D in LDS (once per work-group), bit 1 stages each u tile
//   UNROLL    split of the MFMA k-step loop with the inner part unrolled
//             (tag "unr", sec. 2.4.2)
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
// as long as both operands use it; here j = step*KSTEP + group*KPL + slot.
// The 16x16 result: lane l, register r holds row 4*(l/16) + r, column l%16.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lpx_internal.h"

namespace lpx {
namespace kern {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct ContractArgs {
    const float* __restrict__ D;
    const float* __restrict__ u;
    float* __restrict__ out;
    int64_t E;
    int64_t ntiles;
    int K, Np, nt, nsteps, ldu;
    int np_vec;  // Np % 4 == 0: 16-byte row accesses are aligned
    int e_vec;   // E % 4 == 0
};

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

// D fragment of pair (k, t), step s, read from global memory.
template <int PREC>
__device__ __forceinline__ Frag<PREC> d_frag_global(const ContractArgs& a, int k, int t,
                                                    int s, int lane) {
    const int i = 16 * t + (lane & 15);
    const int ic = i < a.Np ? i : a.Np - 1;
    const int j0 = s * Traits<PREC>::KSTEP + (lane >> 4) * Traits<PREC>::KPL;
    const float* row = a.D + ((int64_t)k * a.Np + ic) * a.Np;
    if constexpr (PREC == LPX_FP32) {
        const float x = row[j0 < a.Np ? j0 : a.Np - 1];
        return make_frag_fp32(i < a.Np && j0 < a.Np ? x : 0.0f);
    } else {
        float v[8];
        load_row8(row, j0, a.Np, a.np_vec, v);
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = i < a.Np ? v[q] : 0.0f;
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
    const int j0 = s * Traits<PREC>::KSTEP + (lane >> 4) * Traits<PREC>::KPL;
    if constexpr (PREC == LPX_FP32) {
        const int jc = j0 < a.Np ? j0 : a.Np - 1;
        const float x = LAYOUT == LPX_ELEMENT_MAJOR ? a.u[ec * a.Np + jc] : a.u[(int64_t)jc * a.E + ec];
        return make_frag_fp32(ev && j0 < a.Np ? x : 0.0f);
    } else {
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

// ------------------------------------------------------------ LDS layout
// [D fragments, operand order: ((k*nt + t)*nsteps + s)*64 + lane]
//   fp32: float; bf16: 16-byte hi plane; bf16x3: hi plane then lo plane
// [u ring: two slots of ldu floats, raw FP32 copies of u tiles]
template <int PREC>
struct Lds {
    static constexpr int DFRAG_BYTES = PREC == LPX_FP32 ? 4 : 16;  // per plane
    static constexpr int PLANES = PREC == LPX_BF16X3 ? 2 : 1;
    static constexpr int UELEM_BYTES = PREC == LPX_FP32 ? 4 : 2;
};

template <int PREC>
__device__ __forceinline__ Frag<PREC> d_frag_lds(const unsigned char* lds, int64_t nfrag,
                                                 int idx) {
    if constexpr (PREC == LPX_FP32) {
        return {reinterpret_cast<const float*>(lds)[idx]};
    } else if constexpr (PREC == LPX_BF16) {
        return {reinterpret_cast<const bf16x8*>(lds)[idx]};
    } else {
        const bf16x8* p = reinterpret_cast<const bf16x8*>(lds);
        return {p[idx], p[nfrag + idx]};
    }
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
// two-slot LDS ring:
//   element-major: the contiguous run u[e0 .. e0+nvalid)[0 .. Np), so
//                  element r, column j sits at r*Np + j;
//   DOF-major:     the Np row segments u[j][e0 .. e0+TILE_E), so column j,
//                  element r sits at j*TILE_E + r.
// A slot has slack past the tile so that reads of padding columns
// (j >= Np, up to the next multiple of 32) stay inside it; those values are
// replaced by zero with a select, never multiplied.  Compute waves convert
// what they read to the operand precision.
template <int PREC, int LAYOUT, int TILE_E>
__device__ __forceinline__ Frag<PREC> u_frag_lds(const float* ut, int Np, bool np_vec, int row0,
                                                 int s, int lane) {
    const int r = row0 + (lane & 15);
    const int j0 = s * Traits<PREC>::KSTEP + (lane >> 4) * Traits<PREC>::KPL;
    if constexpr (PREC == LPX_FP32) {
        const float x = LAYOUT == LPX_ELEMENT_MAJOR ? ut[r * Np + j0] : ut[j0 * TILE_E + r];
        return {j0 < Np ? x : 0.0f};
    } else {
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
                v[t] = LAYOUT == LPX_ELEMENT_MAJOR ? ut[r * Np + j0 + t] : ut[(j0 + t) * TILE_E + r];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = j0 + t < Np ? v[t] : 0.0f;
        return make_frag8<PREC>(v);
    }
}

// Loader waves.  A tile is cut into 16-byte chunks; chunk c goes to slot
// offset 16c bytes.  Loader wave lw (of NLW) holds chunks
// c = lane + 64 * (lw + NLW * q), q < PER_LANE, in registers from one
// iteration to the next, so its global loads are in flight while the
// compute waves work on the previous tile.  Loader waves issue no global
// stores, so their waits cover their own loads only.
//   element-major: chunk c = floats 4c..4c+3 of the run of nvalid*Np floats;
//   DOF-major:     chunk c = row j = c / (TILE_E/4), columns
//                  4*(c % (TILE_E/4)) .. +3.
template <int TILE_E, int NTMAX, int NLW>
struct Loader {
    static constexpr int CHUNKS = TILE_E * 16 * NTMAX / 4;  // upper bound per tile
    static constexpr int PER_LANE = (CHUNKS + 64 * NLW - 1) / (64 * NLW);
};

// Number of chunks of a tile with nvalid elements.
template <int LAYOUT, int TILE_E>
__device__ __forceinline__ int tile_chunks(const ContractArgs& a, int nvalid) {
    return LAYOUT == LPX_ELEMENT_MAJOR ? (nvalid * a.Np + 3) / 4 : a.Np * (TILE_E / 4);
}

template <int LAYOUT, int TILE_E, int NTMAX, int NLW>
__device__ __forceinline__ void loader_fetch(const ContractArgs& a, int64_t e0, int nvalid, int lw,
                                             int lane, f4 (&v)[Loader<TILE_E, NTMAX, NLW>::PER_LANE]) {
    constexpr int PL = Loader<TILE_E, NTMAX, NLW>::PER_LANE;
    const int nch = tile_chunks<LAYOUT, TILE_E>(a, nvalid);
    if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
        const float* src = a.u + e0 * a.Np;  // 16-byte aligned: e0 % 16 == 0
        const int nflat = nvalid * a.Np;
        if (nflat % 4 == 0) {  // uniform: every chunk below nch is whole
#pragma unroll
            for (int q = 0; q < PL; ++q) {
                int c = lane + 64 * (lw + NLW * q);
                c = c < nch ? c : nch - 1;  // the duplicate is not stored
                v[q] = *reinterpret_cast<const f4*>(src + 4 * c);
            }
        } else {  // the last tile of an odd-sized run
            for (int q = 0; q < PL; ++q) {
                const int c = lane + 64 * (lw + NLW * q);
                f4 x = {0.f, 0.f, 0.f, 0.f};
                for (int t = 0; t < 4; ++t)
                    if (4 * c + t < nflat) x[t] = src[4 * c + t];
                v[q] = x;
            }
        }
    } else {
        constexpr int CPR = TILE_E / 4;
        if (a.e_vec) {  // uniform: E % 4 == 0, so nvalid % 4 == 0 and rows are aligned
#pragma unroll
            for (int q = 0; q < PL; ++q) {
                int c = lane + 64 * (lw + NLW * q);
                c = c < nch ? c : nch - 1;
                const int j = c / CPR;
                int col = 4 * (c % CPR);
                col = col < nvalid ? col : nvalid - 4;  // columns >= nvalid are never used
                v[q] = *reinterpret_cast<const f4*>(a.u + (int64_t)j * a.E + e0 + col);
            }
        } else {
            for (int q = 0; q < PL; ++q) {
                const int c = lane + 64 * (lw + NLW * q);
                const int j = c / CPR, col = 4 * (c % CPR);
                f4 x = {0.f, 0.f, 0.f, 0.f};
                if (c < nch)
                    for (int t = 0; t < 4; ++t)
                        if (col + t < nvalid) x[t] = a.u[(int64_t)j * a.E + e0 + col + t];
                v[q] = x;
            }
        }
    }
}

template <int LAYOUT, int TILE_E, int NTMAX, int NLW>
__device__ __forceinline__ void loader_put(const ContractArgs& a, float* ut, int nvalid, int lw,
                                           int lane,
                                           const f4 (&v)[Loader<TILE_E, NTMAX, NLW>::PER_LANE]) {
    constexpr int PL = Loader<TILE_E, NTMAX, NLW>::PER_LANE;
    const int nch = tile_chunks<LAYOUT, TILE_E>(a, nvalid);
#pragma unroll
    for (int q = 0; q < PL; ++q) {
        const int c = lane + 64 * (lw + NLW * q);
        if (c < nch) reinterpret_cast<f4*>(ut)[c] = v[q];
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
    const int64_t nfrag = (int64_t)a.K * a.nt * a.nsteps * 64;
    for (int64_t base = 0; base < nfrag; base += (int64_t)NTHREADS * U) {
        Frag<PREC> f[U];
#pragma unroll
        for (int b = 0; b < U; ++b) {
            int64_t idx = base + tid + (int64_t)NTHREADS * b;
            idx = idx < nfrag ? idx : nfrag - 1;  // clamped: the duplicate is not stored
            const int l = (int)(idx & 63);
            const int rest = (int)(idx >> 6);
            const int s = rest % a.nsteps;
            const int p = rest / a.nsteps;
            const int k = p / a.nt;
            const int t = p - k * a.nt;
            f[b] = d_frag_global<PREC>(a, k, t, s, l);
        }
#pragma unroll
        for (int b = 0; b < U; ++b) {
            const int64_t idx = base + tid + (int64_t)NTHREADS * b;
            if (idx < nfrag) d_frag_store_lds<PREC>(lds, nfrag, (int)idx, f[b]);
        }
    }
}

// Write-back of one chunk of a wave's pairs (p = pc + q*WPE, q < PMAX).
template <int LAYOUT, int PMAX, int WPE>
__device__ __forceinline__ void store_pairs(const ContractArgs& a, const f4 (&acc)[PMAX], int pc,
                                            int64_t eb0, int lane) {
    const int npairs = a.K * a.nt;
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
        const int p = pc + q * WPE;
        if (p >= npairs) continue;
        const int k = p / a.nt, t = p - (p / a.nt) * a.nt;
        if constexpr (LAYOUT == LPX_ELEMENT_MAJOR) {
            const int64_t e = eb0 + (lane & 15);
            const int i0 = 16 * t + 4 * (lane >> 4);
            if (e < a.E && i0 < a.Np) {
                float* dst = a.out + ((int64_t)k * a.E + e) * a.Np + i0;
                if (a.np_vec) {
                    *reinterpret_cast<f4*>(dst) = acc[q];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (i0 + r < a.Np) dst[r] = acc[q][r];
                }
            }
        } else {
            const int i = 16 * t + (lane & 15);
            const int64_t e = eb0 + 4 * (lane >> 4);
            if (i < a.Np && e < a.E) {
                float* dst = a.out + ((int64_t)k * a.Np + i) * a.E + e;
                if (a.e_vec) {
                    *reinterpret_cast<f4*>(dst) = acc[q];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (e + r < a.E) dst[r] = acc[q][r];
                }
            }
        }
    }
}

// One wave's share of a 16-element block starting at element eb0: the
// (k, i-block) pairs p = part, part + WPE, ... (WPE waves share a block);
// for each, the MFMA chain over the k-steps of j, then the write-back.
// D fragments come from LDS (PF_D) or global memory; u fragments from the
// staged tile `ut` at row `row0` (PF_U) or global memory.  The summation
// order of every output depends only on PREC: all records of a precision
// give bit-identical results.
template <int PREC, int LAYOUT, int NTMAX, bool PF_D, bool PF_U, int TILE_E, int WPE, int UNROLL>
__device__ __forceinline__ void block_compute(const ContractArgs& a, const unsigned char* lds,
                                              const float* ut, int row0, int64_t eb0, int part,
                                              int lane) {
    constexpr int PMAX = (3 * NTMAX + WPE - 1) / WPE;  // pairs held per wave
    const int npairs = a.K * a.nt;
    const int64_t nfrag = (int64_t)npairs * a.nsteps * 64;
    for (int pc = part; pc < npairs; pc += WPE * PMAX) {
        f4 acc[PMAX];
        int pk[PMAX], pt[PMAX];
#pragma unroll
        for (int q = 0; q < PMAX; ++q) {
            acc[q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            const int p = pc + q * WPE;
            pk[q] = p / a.nt;
            pt[q] = p - pk[q] * a.nt;
        }
        auto step = [&](int s) {
            Frag<PREC> uf;
            if constexpr (PF_U)
                uf = u_frag_lds<PREC, LAYOUT, TILE_E>(ut, a.Np, a.np_vec, row0, s, lane);
            else
                uf = u_frag_global<PREC, LAYOUT>(a, eb0, s, lane);
#pragma unroll
            for (int q = 0; q < PMAX; ++q) {
                const int p = pc + q * WPE;
                if (p < npairs) {
                    Frag<PREC> df;
                    if constexpr (PF_D)
                        df = d_frag_lds<PREC>(lds, nfrag, (p * a.nsteps + s) * 64 + lane);
                    else
                        df = d_frag_global<PREC>(a, pk[q], pt[q], s, lane);
                    if constexpr (LAYOUT == LPX_ELEMENT_MAJOR)
                        acc[q] = mma(df, uf, acc[q]);  // rows i, columns e
                    else
                        acc[q] = mma(uf, df, acc[q]);  // rows e, columns i
                }
            }
        };
        int s = 0;
        for (; s + UNROLL <= a.nsteps; s += UNROLL) {
#pragma unroll
            for (int uu = 0; uu < UNROLL; ++uu) step(s + uu);
        }
        for (; s < a.nsteps; ++s) step(s);
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
    Frag<PREC> f[PMAX][NS];
};

template <int PREC, int NTMAX, int WPE>
__device__ __forceinline__ void load_dregs(const ContractArgs& a, int part, int lane,
                                           DRegs<PREC, NTMAX, WPE>& d) {
    using DR = DRegs<PREC, NTMAX, WPE>;
    const int npairs = a.K * a.nt;
#pragma unroll
    for (int q = 0; q < DR::PMAX; ++q) {
        int p = part + q * WPE;
        p = p < npairs ? p : npairs - 1;  // clamped: the duplicate is never used
        const int k = p / a.nt, t = p - (p / a.nt) * a.nt;
#pragma unroll
        for (int s = 0; s < DR::NS; ++s) d.f[q][s] = d_frag_global<PREC>(a, k, t, s, lane);
    }
}

template <int PREC, int LAYOUT, int NTMAX, bool PF_U, int TILE_E, int WPE>
__device__ __forceinline__ void block_compute_dreg(const ContractArgs& a,
                                                   const DRegs<PREC, NTMAX, WPE>& d,
                                                   const float* ut, int row0, int64_t eb0,
                                                   int part, int lane) {
    using DR = DRegs<PREC, NTMAX, WPE>;
    const int npairs = a.K * a.nt;
    f4 acc[DR::PMAX];
#pragma unroll
    for (int q = 0; q < DR::PMAX; ++q) acc[q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < DR::NS; ++s) {
        if (s >= a.nsteps) break;  // uniform
        Frag<PREC> uf;
        if constexpr (PF_U)
            uf = u_frag_lds<PREC, LAYOUT, TILE_E>(ut, a.Np, a.np_vec, row0, s, lane);
        else
            uf = u_frag_global<PREC, LAYOUT>(a, eb0, s, lane);
#pragma unroll
        for (int q = 0; q < DR::PMAX; ++q) {
            if (part + q * WPE < npairs) {
                if constexpr (LAYOUT == LPX_ELEMENT_MAJOR)
                    acc[q] = mma(d.f[q][s], uf, acc[q]);
                else
                    acc[q] = mma(uf, d.f[q][s], acc[q]);
            }
        }
    }
    store_pairs<LAYOUT, DR::PMAX, WPE>(a, acc, part, eb0, lane);
}

// ------------------------------------------------------------ the kernel
// Work-group shape.  Without a staged u tile: four waves per 16-element
// block, splitting its (k, i-block) pairs.  With one: min(4 * TILE_E/16, 8)
// compute waves (so WPE = that / (TILE_E/16) per block) plus NLW loader
// waves that keep the next tile in registers.
template <int TILE_E, int NTMAX, int PREFETCH>
struct Shape {
    static constexpr bool PF_U = (PREFETCH & 2) != 0;
    static constexpr ContractShape CS = contract_shape(TILE_E, NTMAX, PREFETCH);
    static constexpr int NCW = CS.ncw, WPE = CS.wpe, NLW = CS.nlw, THREADS = CS.threads;
};

template <int PREC, int LAYOUT, int NTMAX, int TILE_E, int PREFETCH, int UNROLL>
__global__ __launch_bounds__((Shape<TILE_E, NTMAX, PREFETCH>::THREADS)) void contract_kernel(
    ContractArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    using S = Shape<TILE_E, NTMAX, PREFETCH>;
    constexpr bool PF_D = (PREFETCH & 1) != 0;
    constexpr bool PF_U = S::PF_U;
    constexpr bool D_REG = (PREFETCH & 4) != 0;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t nfrag = (int64_t)a.K * a.nt * a.nsteps * 64;
    float* ring = reinterpret_cast<float*>(
        lds + (PF_D ? nfrag * Lds<PREC>::DFRAG_BYTES * Lds<PREC>::PLANES : 0));
    const int slot_floats = a.ldu;  // ring slot stride (floats)

    if constexpr (PF_D) stage_d<PREC, S::THREADS>(a, lds, tid);

    if constexpr (!PF_U) {
        if constexpr (PF_D) __syncthreads();
        const int eblk = wave / S::WPE, part = wave % S::WPE;
        if constexpr (D_REG) {
            DRegs<PREC, NTMAX, S::WPE> d;
            load_dregs<PREC, NTMAX, S::WPE>(a, part, lane, d);
            for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
                const int64_t e0 = tile * TILE_E;
                if (e0 + 16 * eblk >= a.E) continue;
                block_compute_dreg<PREC, LAYOUT, NTMAX, false, TILE_E, S::WPE>(
                    a, d, nullptr, 0, e0 + 16 * eblk, part, lane);
            }
        } else {
            for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
                const int64_t e0 = tile * TILE_E;
                if (e0 + 16 * eblk >= a.E) continue;  // uniform per wave; no barrier below
                block_compute<PREC, LAYOUT, NTMAX, PF_D, false, TILE_E, S::WPE, UNROLL>(
                    a, lds, nullptr, 0, e0 + 16 * eblk, part, lane);
            }
        }
    } else {
        auto nvalid_of = [&](int64_t tile) {
            const int64_t rest = a.E - tile * TILE_E;
            return (int)(rest < TILE_E ? rest : TILE_E);
        };
        // Loader and compute waves run separate loops with one barrier per
        // tile each, so their registers are never live at the same time.
        if (wave >= S::NCW) {
            const int lw = wave - S::NCW;
            f4 held[Loader<TILE_E, NTMAX, S::NLW>::PER_LANE];
            int64_t tile = blockIdx.x;
            if (tile < a.ntiles) {
                // Prologue: tile 0 into slot 0, tile 1 held in registers.
                loader_fetch<LAYOUT, TILE_E, NTMAX, S::NLW>(a, tile * TILE_E, nvalid_of(tile),
                                                             lw, lane, held);
                loader_put<LAYOUT, TILE_E, NTMAX, S::NLW>(a, ring, nvalid_of(tile), lw, lane,
                                                           held);
                const int64_t t1 = tile + gridDim.x;
                if (t1 < a.ntiles)
                    loader_fetch<LAYOUT, TILE_E, NTMAX, S::NLW>(a, t1 * TILE_E, nvalid_of(t1),
                                                                 lw, lane, held);
            }
            __syncthreads();
            for (int n = 0; tile < a.ntiles; ++n, tile += gridDim.x) {
                const int64_t t1 = tile + gridDim.x, t2 = t1 + gridDim.x;
                if (t1 < a.ntiles) {
                    // slot ^ 1 was last read in the previous iteration
                    loader_put<LAYOUT, TILE_E, NTMAX, S::NLW>(
                        a, ring + ((n & 1) ^ 1) * slot_floats, nvalid_of(t1), lw, lane, held);
                    if (t2 < a.ntiles)
                        loader_fetch<LAYOUT, TILE_E, NTMAX, S::NLW>(a, t2 * TILE_E,
                                                                     nvalid_of(t2), lw, lane, held);
                }
                __syncthreads();  // slot read by the compute waves; slot ^ 1 filled
            }
        } else {
            const int eblk = wave / S::WPE, part = wave % S::WPE;
            if constexpr (D_REG) {
                DRegs<PREC, NTMAX, S::WPE> d;
                load_dregs<PREC, NTMAX, S::WPE>(a, part, lane, d);
                __syncthreads();
                int64_t tile = blockIdx.x;
                for (int n = 0; tile < a.ntiles; ++n, tile += gridDim.x) {
                    if (16 * eblk < nvalid_of(tile))
                        block_compute_dreg<PREC, LAYOUT, NTMAX, true, TILE_E, S::WPE>(
                            a, d, ring + (n & 1) * slot_floats, 16 * eblk,
                            tile * TILE_E + 16 * eblk, part, lane);
                    __syncthreads();
                }
            } else {
                __syncthreads();
                int64_t tile = blockIdx.x;
                for (int n = 0; tile < a.ntiles; ++n, tile += gridDim.x) {
                    if (16 * eblk < nvalid_of(tile))
                        block_compute<PREC, LAYOUT, NTMAX, PF_D, true, TILE_E, S::WPE, UNROLL>(
                            a, lds, ring + (n & 1) * slot_floats, 16 * eblk,
                            tile * TILE_E + 16 * eblk, part, lane);
                    __syncthreads();
                }
            }
        }
    }
}

}  // namespace kern
}  // namespace lpx
