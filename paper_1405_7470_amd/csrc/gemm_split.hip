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
//   2. the main kernel computes a 128 x 128 tile of C per work-group of
//      four waves (each a 64 x 64 quarter of 16 x 16 MFMA blocks), k in
//      slabs of 64.  Slabs are copied global -> LDS with direct loads
//      (global_load_lds_dwordx4, no registers), double-buffered so that the
//      next slab arrives while the current one is multiplied.
//
// LDS slab: 128 rows of 64 bf16 (128 bytes, eight 16-byte columns).  Column
// c of row r is stored at column c ^ ((r >> 1) & 7), so the 16 rows that a
// fragment read touches fall in 16 distinct bank groups.  A loader lane
// writes a fixed LDS position; it fetches the global chunk that belongs
// there.
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

constexpr int TM = 128, TN = 128, TK = 64;
constexpr int SLAB_BYTES = TM * TK * 2;  // one plane of one operand: 16 KiB
static_assert(TM == TN, "A and B slabs share one layout");

constexpr int vmcnt0 = (7 << 4) | (15 << 8);  // s_waitcnt vmcnt(0), other counters untouched

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

// 16-byte column position of (row r, column c) in a slab.
__device__ __forceinline__ int slab_pos(int r, int c) { return r * 8 + (c ^ ((r >> 1) & 7)); }

// Issues this wave's direct loads of one plane of one operand's slab:
// 1024 chunks, four instructions per wave.  rows0: first global row of the
// tile, nrows: rows in the matrix (rows past it read the last row).
__device__ __forceinline__ void load_slab(const __bf16* plane, int64_t rows0, int64_t nrows,
                                          int64_t Kp, int64_t k0, unsigned char* slab, int wave,
                                          int lane) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int blk = wave * 4 + q;  // 64 positions per instruction
        const int p = blk * 64 + lane;
        const int r = p >> 3;
        const int c = (p & 7) ^ ((r >> 1) & 7);
        int64_t row = rows0 + r;
        row = row < nrows ? row : nrows - 1;
        const __bf16* src = plane + row * Kp + k0 + 8 * c;
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(src),
                                         (lds_void*)(slab + blk * 1024), 16, 0, 0);
    }
}

__device__ __forceinline__ bf16x8 frag(const unsigned char* slab, int r0, int s2, int lane) {
    const int r = r0 + (lane & 15);
    const int c = 4 * s2 + (lane >> 4);
    return *reinterpret_cast<const bf16x8*>(slab + 16 * slab_pos(r, c));
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

template <int PLANES>
__global__ __launch_bounds__(256) void gemm_split_kernel(Args g) {
    extern __shared__ __align__(16) unsigned char lds[];
    // stage s: A planes then B planes, SLAB_BYTES each
    constexpr int STAGE = 2 * PLANES * SLAB_BYTES;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int64_t tm, tn;
    tile_of(blockIdx.x, gridDim.x, g.tiles_n, &tm, &tn);
    const int64_t m0 = tm * TM, n0 = tn * TN;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

    auto issue = [&](int64_t kt) {
        unsigned char* st = lds + (kt & 1) * STAGE;
#pragma unroll
        for (int p = 0; p < PLANES; ++p) {
            load_slab(g.A + p * g.M * g.Kp, m0, g.M, g.Kp, kt * TK, st + p * SLAB_BYTES, wave,
                      lane);
            load_slab(g.B + p * g.N * g.Kp, n0, g.N, g.Kp, kt * TK,
                      st + (PLANES + p) * SLAB_BYTES, wave, lane);
        }
    };

    f4 acc[4][4];  // [n block][m block]
#pragma unroll
    for (int bn = 0; bn < 4; ++bn)
#pragma unroll
        for (int bm = 0; bm < 4; ++bm) acc[bn][bm] = f4{0.f, 0.f, 0.f, 0.f};

    const int64_t nk = g.Kp / TK;
    issue(0);
    __builtin_amdgcn_s_waitcnt(vmcnt0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        // the next slab goes to the other stage, last read in iteration kt-1
        if (kt + 1 < nk) issue(kt + 1);
        const unsigned char* st = lds + (kt & 1) * STAGE;
#pragma unroll
        for (int s2 = 0; s2 < TK / 32; ++s2) {
            bf16x8 ah[4], bh[4], al[4], bl[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                ah[b] = frag(st, wm + 16 * b, s2, lane);
                bh[b] = frag(st + PLANES * SLAB_BYTES, wn + 16 * b, s2, lane);
                if constexpr (PLANES == 2) {
                    al[b] = frag(st + SLAB_BYTES, wm + 16 * b, s2, lane);
                    bl[b] = frag(st + 3 * SLAB_BYTES, wn + 16 * b, s2, lane);
                }
            }
#pragma unroll
            for (int bn = 0; bn < 4; ++bn)
#pragma unroll
                for (int bm = 0; bm < 4; ++bm) {
                    f4 c = acc[bn][bm];
                    if constexpr (PLANES == 2) {
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[bn], ah[bm], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[bn], al[bm], c, 0, 0, 0);
                    }
                    acc[bn][bm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[bn], ah[bm], c, 0, 0, 0);
                }
        }
        __builtin_amdgcn_s_waitcnt(vmcnt0);  // slab kt+1 has landed
        __syncthreads();                      // ... for every wave; stage kt is free
    }

    // acc[bn][bm]: lane holds C[m][n .. n+3], m = wm + 16 bm + lane%16,
    // n = wn + 16 bn + 4 (lane/16)
    const bool vec = (g.ldc % 4) == 0;
#pragma unroll
    for (int bn = 0; bn < 4; ++bn)
#pragma unroll
        for (int bm = 0; bm < 4; ++bm) {
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

template <int PLANES>
lpx_status run(const lpx_gemm_desc& d, hipStream_t st) {
    const int64_t Kp = round_up(d.K, TK);
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
    const int lds = 2 * 2 * PLANES * SLAB_BYTES;
    auto fn = &gemm_split_kernel<PLANES>;
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

// Precondition: validated descriptor with M, N > 0, precision bf16 or bf16x3.
lpx_status launch_gemm_split(const lpx_gemm_desc& d, int precision, void* stream) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if ((d.M + 127) / 128 * ((d.N + 127) / 128) > 0x7fffffff)
        return set_error(LPX_ERR_UNSUPPORTED, "GEMM grid too large");
    return precision == LPX_BF16 ? gsplit::run<1>(d, st) : gsplit::run<2>(d, st);
}

}  // namespace lpx
