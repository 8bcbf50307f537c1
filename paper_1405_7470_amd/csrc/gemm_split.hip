// GEMM C = A B in BF16 or split-precision bf16x3 on pre-split operands.
//
// The degenerate case of the contraction (sec. 2.1, Table 1's "sgemm")
// for the two reduced precisions, with the operand conversion hoisted out
// of the k loop (the split-precision step, applied once per call to both
// operands as it is to D in the contraction):
//
//   1. split kernels write each operand as K-contiguous bf16 planes (hi,
//      and lo = bf16(x - hi) for bf16x3) zero-padded to Kp = K rounded up
//      to 64: A as [M][Kp], B transposed as [N][Kp];
//   2. the main kernel computes a TM x TN tile of C per work-group of four
//      waves (2 x 2, each a TM/2 x TN/2 quarter of 16 x 16 MFMA blocks), k
//      in slabs of TK.  Slabs are copied global -> LDS with direct loads
//      (global_load_lds_dwordx4, no registers), double-buffered so that the
//      next slab arrives while the current one is multiplied.  Built: 128 x
//      128 x 64, and 256 x 256 / 256 x 128 with TK = 64 (BF16) or 32
//      (bf16x3, two planes per operand).  A wave tile of W x W reads
//      2W x TK bf16 from LDS per W x W x TK MFMA work, so the 128 x 128 wave
//      tile of the 256 x 256 tiling needs half the LDS bandwidth per MFMA of
//      the 64 x 64 one (which reads LDS at the full LDS rate at peak MFMA).
//
// LDS slab: rows of TK bf16 (TK/8 16-byte columns).  Column c of row r is
// stored at column c ^ swz(r), swz(r) = (r >> 1) & 7 for 128-byte rows and
// (r >> 2) & 3 for 64-byte rows, so the 16 rows that a fragment read
// touches fall in distinct bank groups.  A loader lane writes a fixed LDS
// position; it fetches the global chunk that belongs there.
//
// MFMA roles: n on the MFMA row axis (B^T plane as the first operand), so
// each lane ends with four consecutive n of one row m: one 16-byte store.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <cstring>
#include <map>

#include "lpx_internal.h"

namespace lpx {
namespace gsplit {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int KPAD = 64;  // planes are zero-padded to a multiple of 64 columns

// s_waitcnt immediate for vmcnt(n), 0 <= n <= 63, other counters untouched
// (vmcnt bits 3:0 and 15:14, expcnt 6:4 at 7, lgkmcnt 11:8 at 15)
constexpr int vmcnt(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// ------------------------------------------------------------ split kernels
// A (M x K, row stride lda) -> planes [M][Kp]; one thread per 8 columns.
template <int PLANES>
__global__ __launch_bounds__(256) void split_rows(const float* __restrict__ A, int64_t M,
                                                  int64_t K, int64_t lda, int64_t Kp,
                                                  __bf16* __restrict__ out) {
    const int64_t nc = Kp / 8;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= M * nc) return;
    const int64_t m = t / nc, k0 = (t % nc) * 8;
    const float* row = A + m * lda;
    float x[8];
    if ((lda & 3) == 0 && k0 + 8 <= K) {  // two 16-byte loads (rows 16-byte aligned)
        const f4 a = *reinterpret_cast<const f4*>(row + k0);
        const f4 b = *reinterpret_cast<const f4*>(row + k0 + 4);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            x[q] = a[q];
            x[q + 4] = b[q];
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) x[q] = k0 + q < K ? row[k0 + q] : 0.0f;
    }
    bf16x8 h, l;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const __bf16 hq = (__bf16)x[q];
        h[q] = hq;
        l[q] = (__bf16)(x[q] - (float)hq);
    }
    *reinterpret_cast<bf16x8*>(out + m * Kp + k0) = h;
    if constexpr (PLANES == 2) *reinterpret_cast<bf16x8*>(out + M * Kp + m * Kp + k0) = l;
}

// B (K x N, row stride ldb) -> transposed planes [N][Kp], through a 64 x 64
// LDS tile so that both the reads (along n) and the writes (along k) are
// contiguous.
template <int PLANES>
__global__ __launch_bounds__(256) void split_transpose(const float* __restrict__ B, int64_t K,
                                                       int64_t N, int64_t ldb, int64_t Kp,
                                                       __bf16* __restrict__ out) {
    __shared__ float tile[64][65];
    const int64_t k0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + 256 * q;
        const int r = e / 64, c = e % 64;  // r: k, c: n
        const int64_t k = k0 + r, n = n0 + c;
        tile[r][c] = (k < K && n < N) ? B[k * ldb + n] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int ch = tid + 256 * q;      // 512 chunks of 8 k
        const int c = ch / 8, r0 = 8 * (ch % 8);  // c: n within the tile
        const int64_t n = n0 + c, k = k0 + r0;
        if (n >= N || k >= Kp) continue;
        bf16x8 h, l;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const float x = tile[r0 + t][c];
            const __bf16 ht = (__bf16)x;
            h[t] = ht;
            l[t] = (__bf16)(x - (float)ht);
        }
        *reinterpret_cast<bf16x8*>(out + n * Kp + k) = h;
        if constexpr (PLANES == 2) *reinterpret_cast<bf16x8*>(out + N * Kp + n * Kp + k) = l;
    }
}

// ------------------------------------------------------------- main kernel
struct Args {
    const __bf16* __restrict__ A;  // PLANES x [M][Kp]
    const __bf16* __restrict__ B;  // PLANES x [N][Kp]
    float* __restrict__ C;
    int64_t M, N, Kp, ldc, tiles_n;
};

// 16-byte column position of (row r, column c) in a slab of CPR columns.
template <int CPR>
__device__ __forceinline__ int slab_pos(int r, int c) {
    static_assert(CPR == 8 || CPR == 4, "slab rows of 64 or 32 bf16");
    return CPR == 8 ? r * 8 + (c ^ ((r >> 1) & 7)) : r * 4 + (c ^ ((r >> 2) & 3));
}

// Issues this wave's direct loads of one plane of one operand's slab (ROWS
// rows of CPR 16-byte chunks).  rows0: first global row of the tile, nrows:
// rows in the matrix (rows past it read the last row).
template <int ROWS, int CPR>
__device__ __forceinline__ void load_slab(const __bf16* plane, int64_t rows0, int64_t nrows,
                                          int64_t Kp, int64_t k0, unsigned char* slab, int wave,
                                          int lane) {
    constexpr int PER_WAVE = ROWS * CPR / (4 * 64);  // 64 positions per instruction
#pragma unroll
    for (int q = 0; q < PER_WAVE; ++q) {
        const int blk = wave * PER_WAVE + q;
        const int p = blk * 64 + lane;
        const int r = p / CPR;
        const int c = CPR == 8 ? (p & 7) ^ ((r >> 1) & 7) : (p & 3) ^ ((r >> 2) & 3);
        int64_t row = rows0 + r;
        row = row < nrows ? row : nrows - 1;
        const __bf16* src = plane + row * Kp + k0 + 8 * c;
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(src),
                                         (lds_void*)(slab + blk * 1024), 16, 0, 0);
    }
}

// The two MFMA shapes.  The B fragment is the MFMA's first operand and the
// A fragment its second, so a lane's accumulator values run along n (four
// consecutive columns of C per 16-byte store) at one row m.
//   16 x 16 x 32: operand lane l holds row l % 16, k 8 (l / 16) .. + 7;
//                 result register r of lane l is (n, m) = (4 (l / 16) + r, l % 16).
//   32 x 32 x 16: operand lane l holds row l % 32, k 8 (l / 32) .. + 7;
//                 result register r of lane l is
//                 (n, m) = (8 (r / 4) + 4 (l / 32) + r % 4, l % 32).
// A single wave per SIMD keeps the 32 x 32 x 16 pipe near full issue rate;
// back-to-back 16 x 16 x 32 MFMAs of one wave do not, so that shape needs two
// waves per SIMD.
typedef float f16v __attribute__((ext_vector_type(16)));
template <int MB>
struct Mma;
template <>
struct Mma<16> {
    typedef f4 acc_t;
    static constexpr int K = 32;
    __device__ static acc_t run(bf16x8 b, bf16x8 a, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a, c, 0, 0, 0);
    }
};
template <>
struct Mma<32> {
    typedef f16v acc_t;
    static constexpr int K = 16;
    __device__ static acc_t run(bf16x8 b, bf16x8 a, acc_t c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(b, a, c, 0, 0, 0);
    }
};

// Operand fragment of MFMA k-step s for rows r0 .. r0 + MB - 1.
template <int CPR, int MB>
__device__ __forceinline__ bf16x8 frag(const unsigned char* slab, int r0, int s, int lane) {
    const int r = r0 + (lane & (MB - 1));
    const int c = (Mma<MB>::K / 8) * s + lane / MB;
    return *reinterpret_cast<const bf16x8*>(slab + 16 * slab_pos<CPR>(r, c));
}

// Work-group -> C tile.  Work-groups are dispatched to the eight XCDs in
// turn (work-group b to XCD b % 8), each with its own L2.  Work-group b gets
// tile t = (b % 8) * (ntiles / 8) + b / 8, so an XCD works through one
// contiguous eighth of the tiles; inside it, tiles go in groups of eight
// tile rows, column by column, so the work-groups resident on one XCD at a
// time cover a square patch of C and share their A rows and B columns in
// that XCD's L2.  (Identity mapping when the tile count is not a multiple
// of 8.)
constexpr int kXcds = 8, kGroupM = 8;
__device__ __forceinline__ void tile_of(int64_t b, int64_t ntiles, int64_t tiles_n, int64_t* tm,
                                        int64_t* tn) {
    int64_t t = b;
    if (ntiles % kXcds == 0) t = (b % kXcds) * (ntiles / kXcds) + b / kXcds;
    const int64_t tiles_m = ntiles / tiles_n;
    const int64_t per_group = kGroupM * tiles_n;
    const int64_t first_m = (t / per_group) * kGroupM;
    const int64_t gsize = tiles_m - first_m < kGroupM ? tiles_m - first_m : kGroupM;
    const int64_t r = t % per_group;
    *tm = first_m + r % gsize;
    *tn = r / gsize;
}

template <int PLANES, int TM, int TN, int TK, int NS>
constexpr int lds_bytes() {
    return NS * PLANES * (TM + TN) * TK * 2;
}

// NS: slabs in the LDS ring; NS - 1 of them are in flight while one is
// multiplied.  MB: MFMA block (16 or 32).
template <int PLANES, int TM, int TN, int TK, int NS, int MB>
__global__ __launch_bounds__(256) void gemm_split_kernel(Args g) {
    extern __shared__ __align__(16) unsigned char lds[];
    using M = Mma<MB>;
    using acc_t = typename M::acc_t;
    constexpr int CPR = TK / 8;                    // 16-byte columns per slab row
    constexpr int A_BYTES = TM * TK * 2, B_BYTES = TN * TK * 2;  // one plane
    constexpr int STAGE = PLANES * (A_BYTES + B_BYTES);
    constexpr int BM = TM / 2 / MB, BN = TN / 2 / MB;  // MFMA blocks per wave quarter
    constexpr int S = TK / M::K;                   // MFMA k-steps per slab
    constexpr int LOADS = PLANES * (TM + TN) * CPR / 256;  // direct loads per wave per slab
    static_assert(NS >= 2 && LOADS * (NS - 2) <= 63, "vmcnt holds at most 63");
    static_assert(BN >= 2 && S >= 1, "two B columns are read ahead");
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int64_t tm, tn;
    tile_of(blockIdx.x, gridDim.x, g.tiles_n, &tm, &tn);
    const int64_t m0 = tm * TM, n0 = tn * TN;
    const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * (TN / 2);

    // stage layout: A planes (hi, lo) then B planes
    auto issue = [&](int64_t kt, int stage) {
        unsigned char* st = lds + stage * STAGE;
#pragma unroll
        for (int p = 0; p < PLANES; ++p) {
            load_slab<TM, CPR>(g.A + p * g.M * g.Kp, m0, g.M, g.Kp, kt * TK, st + p * A_BYTES,
                               wave, lane);
            load_slab<TN, CPR>(g.B + p * g.N * g.Kp, n0, g.N, g.Kp, kt * TK,
                               st + PLANES * A_BYTES + p * B_BYTES, wave, lane);
        }
    };

    acc_t acc[BN][BM];  // [n block][m block]
#pragma unroll
    for (int bn = 0; bn < BN; ++bn)
#pragma unroll
        for (int bm = 0; bm < BM; ++bm)
#pragma unroll
            for (int r = 0; r < MB * MB / 64; ++r) acc[bn][bm][r] = 0.f;

    const int64_t nk = g.Kp / TK;
    // Loads complete in issue order, so vmcnt(LOADS * (NS - 2)) leaves the
    // NS - 2 newest slabs in flight and waits for the older ones; where fewer
    // were issued (the last slabs) the wait is for all of them.
#pragma unroll
    for (int s = 0; s < NS - 1; ++s)
        if (s < nk) issue(s, s);
    if (nk >= NS - 1)
        __builtin_amdgcn_s_waitcnt(vmcnt(LOADS * (NS - 2)));
    else
        __builtin_amdgcn_s_waitcnt(vmcnt(0));
    __syncthreads();
    int cur = 0, nxt = NS - 1;  // ring slots of slab kt and of slab kt + NS - 1
    for (int64_t kt = 0; kt < nk; ++kt) {
        // slab kt + NS - 1 goes to the slot last read in iteration kt - 1
        const bool more = kt + NS - 1 < nk;
        if (more) issue(kt + NS - 1, nxt);
        const unsigned char* st = lds + cur * STAGE;
        // Fragment reads run ahead of the MFMAs that use them: a k-step's A
        // fragments and its first two B columns before the step's first MFMA
        // group, B column bn + 2 before group bn, and the next step's reads
        // during the last two groups.  LDS reads return in order, so each
        // group waits only for its own operands; sched_barrier keeps the
        // scheduler from sinking the reads back to their first use.
        bf16x8 fa[S][PLANES][BM], fb[S][PLANES][BN];
        auto read_a = [&](int s) {
#pragma unroll
            for (int p = 0; p < PLANES; ++p)
#pragma unroll
                for (int b = 0; b < BM; ++b)
                    fa[s][p][b] = frag<CPR, MB>(st + p * A_BYTES, wm + MB * b, s, lane);
        };
        auto read_b = [&](int s, int bn) {
#pragma unroll
            for (int p = 0; p < PLANES; ++p)
                fb[s][p][bn] =
                    frag<CPR, MB>(st + PLANES * A_BYTES + p * B_BYTES, wn + MB * bn, s, lane);
        };
        read_a(0);
        read_b(0, 0);
        read_b(0, 1);
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int bn = 0; bn < BN; ++bn) {
                if (bn + 2 < BN) {
                    read_b(s, bn + 2);
                } else if (s + 1 < S) {
                    if (bn + 2 == BN) {
                        read_a(s + 1);
                    } else {
                        read_b(s + 1, 0);
                        read_b(s + 1, 1);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                // per accumulator: lo(B) hi(A), hi(B) lo(A), then hi(B) hi(A);
                // the passes over bm keep dependent MFMAs BM apart
                if constexpr (PLANES == 2) {
#pragma unroll
                    for (int bm = 0; bm < BM; ++bm)
                        acc[bn][bm] = M::run(fb[s][1][bn], fa[s][0][bm], acc[bn][bm]);
#pragma unroll
                    for (int bm = 0; bm < BM; ++bm)
                        acc[bn][bm] = M::run(fb[s][0][bn], fa[s][1][bm], acc[bn][bm]);
                }
#pragma unroll
                for (int bm = 0; bm < BM; ++bm)
                    acc[bn][bm] = M::run(fb[s][0][bn], fa[s][0][bm], acc[bn][bm]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // slab kt + 1 has landed ...
        if (more)
            __builtin_amdgcn_s_waitcnt(vmcnt(LOADS * (NS - 2)));
        else
            __builtin_amdgcn_s_waitcnt(vmcnt(0));
        __syncthreads();  // ... for every wave, and slot cur is free
        cur = cur + 1 == NS ? 0 : cur + 1;
        nxt = nxt + 1 == NS ? 0 : nxt + 1;
    }

    // acc[bn][bm] register 4 q + t (q < MB * MB / 256): C[m][n + t],
    // m = wm + MB bm + lane % MB, n = wn + MB bn + 8 q + 4 (lane / MB) for
    // MB = 32 (q < 4), n = wn + 16 bn + 4 (lane / 16) for MB = 16 (q = 0)
    const bool vec = (g.ldc % 4) == 0;
#pragma unroll
    for (int bn = 0; bn < BN; ++bn)
#pragma unroll
        for (int bm = 0; bm < BM; ++bm)
#pragma unroll
            for (int q = 0; q < MB * MB / 256; ++q) {
                const int64_t m = m0 + wm + MB * bm + (lane & (MB - 1));
                const int64_t n = n0 + wn + MB * bn + 8 * q + 4 * (lane / MB);
                if (m >= g.M || n >= g.N) continue;
                const f4 v{acc[bn][bm][4 * q], acc[bn][bm][4 * q + 1], acc[bn][bm][4 * q + 2],
                           acc[bn][bm][4 * q + 3]};
                float* dst = g.C + m * g.ldc + n;
                if (vec && n + 4 <= g.N) {
                    *reinterpret_cast<f4*>(dst) = v;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (n + r < g.N) dst[r] = v[r];
                }
            }
}

}  // namespace gsplit

// Stream-ordered workspace comes from a memory pool the library creates
// and owns, one per device, whose release threshold is raised so that freed
// blocks stay in the pool for the next call (otherwise every call would pay
// for a fresh allocation after each synchronisation).  The device's default
// pool, which other code in the process may use, is left untouched.
namespace {
std::mutex g_pool_mu;
std::map<int, hipMemPool_t> g_pools;
}  // namespace

static lpx_status library_pool(hipMemPool_t* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(LPX_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(g_pool_mu);
    auto it = g_pools.find(dev);
    if (it != g_pools.end()) {
        *out = it->second;
        return LPX_OK;
    }
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof props);
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    e = hipMemPoolCreate(&pool, &props);
    uint64_t keep = UINT64_MAX;
    if (e == hipSuccess) e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    if (e != hipSuccess)
        return set_error(LPX_ERR_HIP, "library memory pool: %s", hipGetErrorString(e));
    g_pools[dev] = pool;
    *out = pool;
    return LPX_OK;
}

lpx_status workspace_alloc(void** p, size_t bytes, void* stream, const char* what) {
    hipMemPool_t pool = nullptr;
    lpx_status s = library_pool(&pool);
    if (s != LPX_OK) return s;
    hipError_t e = hipMallocFromPoolAsync(p, bytes, pool, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(LPX_ERR_HIP, "%s workspace: %s", what, hipGetErrorString(e));
    return LPX_OK;
}

namespace gsplit {

template <int PLANES, int TM, int TN, int TK, int NS, int MB>
lpx_status run(const lpx_gemm_desc& d, hipStream_t st) {
    const int64_t Kp = round_up(d.K, KPAD);
    const int64_t abytes = (int64_t)PLANES * d.M * Kp * 2, bbytes = (int64_t)PLANES * d.N * Kp * 2;
    void* ws = nullptr;
    lpx_status ks = workspace_alloc(&ws, (size_t)(abytes + bbytes), st, "GEMM");
    if (ks != LPX_OK) return ks;
    hipError_t e;
    __bf16* As = static_cast<__bf16*>(ws);
    __bf16* Bs = reinterpret_cast<__bf16*>(static_cast<unsigned char*>(ws) + abytes);
    const int64_t na = d.M * (Kp / 8);
    hipLaunchKernelGGL(split_rows<PLANES>, dim3((unsigned)ceil_div(na, 256)), dim3(256), 0, st,
                       d.A, d.M, d.K, d.lda, Kp, As);
    hipLaunchKernelGGL(split_transpose<PLANES>,
                       dim3((unsigned)ceil_div(d.N, 64), (unsigned)ceil_div(Kp, 64)), dim3(256), 0,
                       st, d.B, d.K, d.N, d.ldb, Kp, Bs);
    Args a{As, Bs, d.C, d.M, d.N, Kp, d.ldc, ceil_div(d.N, TN)};
    constexpr int lds = lds_bytes<PLANES, TM, TN, TK, NS>();
    static_assert(lds <= 160 * 1024, "slabs must fit in LDS");
    auto fn = &gemm_split_kernel<PLANES, TM, TN, TK, NS, MB>;
    if (lds > 64 * 1024) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) {
            (void)hipFreeAsync(ws, st);
            return set_error(LPX_ERR_HIP, "hipFuncSetAttribute: %s", hipGetErrorString(e));
        }
    }
    const int64_t grid = ceil_div(d.M, TM) * a.tiles_n;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(256), (size_t)lds, st, a);
    e = hipGetLastError();
    hipError_t ef = hipFreeAsync(ws, st);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return set_error(LPX_ERR_HIP, "GEMM launch: %s", hipGetErrorString(e));
    return LPX_OK;
}

}  // namespace gsplit

bool gemm_split_tiling(int precision, int tm, int tn, int tk) {
    if (precision == LPX_FP32) return false;
    if (tm == 128 && tn == 128 && tk == 64) return true;
    if (tm != 256) return false;
    if (precision == LPX_BF16) return (tn == 256 && (tk == 32 || tk == 64)) || (tn == 128 && tk == 64);
    return (tn == 256 || tn == 128) && tk == 32;
}

// Precondition: validated descriptor with M, N > 0, K > 0, a tiling that
// gemm_split_tiling accepts.
lpx_status launch_gemm_split(const lpx_gemm_desc& d, int precision, int tm, int tn, int tk,
                             void* stream) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (ceil_div(d.M, tm) * ceil_div(d.N, tn) > 0x7fffffff)
        return set_error(LPX_ERR_UNSUPPORTED, "GEMM grid too large");
    const bool x3 = precision == LPX_BF16X3;
    if (tm == 128) return x3 ? gsplit::run<2, 128, 128, 64, 2, 32>(d, st) : gsplit::run<1, 128, 128, 64, 2, 16>(d, st);
    if (x3) return tn == 256 ? gsplit::run<2, 256, 256, 32, 2, 32>(d, st) : gsplit::run<2, 256, 128, 32, 3, 32>(d, st);
    if (tn == 128) return gsplit::run<1, 256, 128, 64, 3, 32>(d, st);
    return tk == 32 ? gsplit::run<1, 256, 256, 32, 4, 32>(d, st) : gsplit::run<1, 256, 256, 64, 2, 32>(d, st);
}

}  // namespace lpx
