// Ragged batch of contractions in one persistent, graph-captured launch.
//
// Each instance i (its own K, Np, E, pointers) is cut into element tiles;
// the tiles of all instances form one list, largest instances first
// (longest-processing-time order, cost K*Np^2*E).
//
// Staged kernel (the default): 32-element tiles dealt round-robin to the
// persistent work-groups (work-group w takes tiles w, w + G, w + 2G, ...,
// which spreads every instance over all of them).  Each work-group runs the
// contraction's staged pipeline -- loader waves filling a four-slot LDS ring
// of u tiles with direct global-to-LDS loads, eight compute waves (D
// fragments from global memory, L2-resident), four store waves writing the
// previous tile's staged output with contiguous stores -- and every wave
// follows the instance table with its own cursor (tiles of a work-group
// come in increasing order, so the cursor only moves forward).
//
// Direct kernel (when the staged rings do not fit in LDS): 16-element tiles
// pulled in chunks from one atomic counter by four-wave work-groups that
// read u straight from global memory, D staged in LDS when it fits.
//
// Both run the same per-block MFMA routine as lpx_contract, so every output
// is bit-identical to a separate lpx_contract call of the same precision.
// The kernel (after a one-thread counter reset for the direct kernel; no
// memset node) is captured once into a HIP graph on a library-owned stream;
// lpx_batch_submit replays it on the caller's stream after copying the
// (possibly updated) descriptor table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "contract_kernels.h"

namespace lpx {
namespace batchk {

constexpr int kThreadsB = 256;
constexpr int kChunk = 8;                         // tiles per counter fetch (direct kernel)
constexpr int64_t kLdsBudget = 48 * 1024;         // D staging budget per work-group (direct)
constexpr int kTileS = 32;                        // staged kernel: elements per tile
constexpr int kPfS = 10;                          // staged u tile + staged output, D global

struct Item {
    kern::ContractArgs a;
    int64_t tile_begin;  // first global tile index of this instance
    int d_lds;           // stage D in LDS for this instance
    int pad;
};

struct BatchArgs {
    const Item* __restrict__ items;
    unsigned long long* counter;
    int64_t total_tiles;
    int n;
    int ldu, ldo;  // staged kernel: u and output ring slot strides (floats)
};

__global__ void reset_counter(unsigned long long* c) { *c = 0ull; }

template <int PREC, int LAYOUT, int NTMAX>
__global__ __launch_bounds__(kThreadsB) void batch_kernel(BatchArgs b) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ long long s_t0;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // scalar: uniform per wave
    int cur = -1;
    for (;;) {
        if (tid == 0) s_t0 = (long long)atomicAdd(b.counter, (unsigned long long)kChunk);
        __syncthreads();
        const long long tv = s_t0;  // the same value in every lane: make it scalar
        const int64_t t0 = ((int64_t)__builtin_amdgcn_readfirstlane((int)(tv >> 32)) << 32) |
                           (uint32_t)__builtin_amdgcn_readfirstlane((int)(tv & 0xffffffff));
        __syncthreads();  // every thread has read s_t0 before it is rewritten
        if (t0 >= b.total_tiles) break;  // uniform: all waves leave together
        const int64_t t1 = t0 + kChunk < b.total_tiles ? t0 + kChunk : b.total_tiles;
        for (int64_t t = t0; t < t1; ++t) {
            int lo = 0, hi = b.n - 1;  // last instance with tile_begin <= t
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (b.items[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
            }
            const kern::ContractArgs a = b.items[lo].a;
            const bool dl = b.items[lo].d_lds != 0;
            if (lo != cur) {
                cur = lo;
                if (dl) {
                    __syncthreads();  // the previous instance's D is no longer read
                    kern::stage_d<PREC, kThreadsB>(a, lds, tid);
                    __syncthreads();
                }
            }
            const int64_t eb0 = (t - b.items[lo].tile_begin) * 16;
            constexpr int CAP = kern::pmax_cap<NTMAX, 4>();
            kern::with_pmax<CAP, 4, PREC == LPX_FP32 ? 2 : 0>(a.nrb, [&](auto pm) {
                constexpr int P = decltype(pm)::value;
                if (dl)
                    kern::block_compute<PREC, LAYOUT, NTMAX, true, false, 16, 4, 2, false, true, P>(
                        a, lds, nullptr, 0, eb0, wave, lane);
                else  // D arranged in global memory
                    kern::block_compute<PREC, LAYOUT, NTMAX, true, false, 16, 4, 2, false, true, P>(
                        a, a.Darr, nullptr, 0, eb0, wave, lane);
            });
        }
    }
}

// D of every instance in MFMA operand order, written to its slice of the
// batch's arrangement buffer (the first node of the graph, so updated D
// pointers are followed on every replay).
template <int PREC>
__global__ __launch_bounds__(kern::kArrangeThreads) void arrange_all(const Item* __restrict__ items,
                                                                    int n) {
    for (int i = blockIdx.y; i < n; i += gridDim.y) {
        const kern::ContractArgs a = items[i].a;
        kern::stage_d<PREC, kern::kArrangeThreads * kern::kArrangeBlocks>(
            a, const_cast<unsigned char*>(a.Darr),
            blockIdx.x * kern::kArrangeThreads + threadIdx.x);
    }
}

// Instance of tile t, starting the search at instance `cur` (a wave's tiles
// come in increasing order).
__device__ __forceinline__ int advance(const Item* items, int n, int64_t t, int cur) {
    while (cur + 1 < n && items[cur + 1].tile_begin <= t) ++cur;
    return cur;
}

template <int NTMAX>
using ShapeS = kern::Shape<kTileS, NTMAX, kPfS>;

template <int PREC, int LAYOUT, int NTMAX>
__global__ __launch_bounds__((ShapeS<NTMAX>::THREADS)) void batch_staged(BatchArgs b) {
    using S = ShapeS<NTMAX>;
    static_assert(S::BPW == 1, "one block per compute wave and tile");
    extern __shared__ __align__(16) unsigned char lds[];
    float* ring = reinterpret_cast<float*>(lds);
    float* oring = ring + 4 * b.ldu;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // scalar: uniform per wave
    const int64_t t0 = blockIdx.x, g = gridDim.x;
    const int64_t nmine = t0 < b.total_tiles ? (b.total_tiles - 1 - t0) / g + 1 : 0;
    const int64_t niter = nmine + 1;  // store waves trail by one tile
    struct Tile {
        int inst, nvalid;
        int64_t e0;
    };
    auto tile_at = [&](int64_t n, int& cur) {
        const int64_t t = t0 + n * g;
        cur = advance(b.items, b.n, t, cur);
        const int64_t e0 = (t - b.items[cur].tile_begin) * kTileS;
        const int64_t rest = b.items[cur].a.E - e0;
        return Tile{cur, (int)(rest < kTileS ? rest : kTileS), e0};
    };
    int cur = 0;
    if (wave >= S::NCW + S::NLW) {
        const int sw = wave - S::NCW - S::NLW;
        __syncthreads();
        for (int64_t n = 0; n < niter; ++n) {
            if (n >= 1) {
                const Tile tt = tile_at(n - 1, cur);
                kern::store_tile<LAYOUT, kTileS, S::NSW>(b.items[tt.inst].a,
                                                         oring + ((n - 1) & 1) * b.ldo, tt.e0,
                                                         tt.nvalid, sw, lane);
            }
            __syncthreads();
        }
    } else if (wave >= S::NCW) {
        const int lw = wave - S::NCW;
        kern::loader_loop<kern::Loader<kTileS, NTMAX, S::NLW>::PER_LANE>(
            nmine, niter, [&](int64_t n) {
                const Tile tt = tile_at(n, cur);
                return kern::loader_issue<LAYOUT, kTileS, NTMAX, S::NLW>(
                    b.items[tt.inst].a, ring + (n & 3) * b.ldu, tt.e0, tt.nvalid, lw, lane);
            });
    } else {
        const int row0 = 16 * (wave / S::WPE), part = wave % S::WPE;
        __syncthreads();
        for (int64_t n = 0; n < niter; ++n) {
            if (n < nmine) {
                const Tile tt = tile_at(n, cur);
                const kern::ContractArgs& a = b.items[tt.inst].a;
                if (row0 < tt.nvalid) {
                    // the instance's own row-block count: small instances in
                    // a batch built for Np up to 16 * NTMAX run no duplicate
                    // MFMA chains (every size for FP32)
                    constexpr int CAP = kern::pmax_cap<NTMAX, S::WPE>();
                    kern::with_pmax<CAP, S::WPE, PREC == LPX_FP32 ? 2 : 0>(a.nrb, [&](auto pm) {
                        auto run = [&](auto mask) {
                            // D from its arrangement in global memory
                            kern::block_compute<PREC, LAYOUT, NTMAX, true, true, kTileS, S::WPE,
                                                2, true, decltype(mask)::value,
                                                decltype(pm)::value>(
                                a, a.Darr, ring + (n & 3) * b.ldu, row0, tt.e0 + row0, part,
                                lane, oring + (n & 1) * b.ldo);
                        };
                        if (PREC == LPX_FP32 && a.np_vec)  // uniform
                            run(std::false_type());
                        else
                            run(std::true_type());
                    });
                }
            }
            __syncthreads();
        }
    }
}

using BatchFn = void (*)(BatchArgs);

template <int PREC, bool STAGED, int LAYOUT, int NTMAX>
BatchFn kernel_of() {
    if constexpr (STAGED)
        return &batch_staged<PREC, LAYOUT, NTMAX>;
    else
        return &batch_kernel<PREC, LAYOUT, NTMAX>;
}

template <int PREC, bool STAGED>
BatchFn pick(int layout, int ntmax) {
    if (layout == LPX_ELEMENT_MAJOR) {
        if (ntmax == 2) return kernel_of<PREC, STAGED, LPX_ELEMENT_MAJOR, 2>();
        if (ntmax == 4) return kernel_of<PREC, STAGED, LPX_ELEMENT_MAJOR, 4>();
        return kernel_of<PREC, STAGED, LPX_ELEMENT_MAJOR, 8>();
    }
    if (ntmax == 2) return kernel_of<PREC, STAGED, LPX_DOF_MAJOR, 2>();
    if (ntmax == 4) return kernel_of<PREC, STAGED, LPX_DOF_MAJOR, 4>();
    return kernel_of<PREC, STAGED, LPX_DOF_MAJOR, 8>();
}

template <bool STAGED>
BatchFn pick_any(int precision, int layout, int ntmax) {
    return precision == LPX_FP32 ? pick<LPX_FP32, STAGED>(layout, ntmax)
         : precision == LPX_BF16 ? pick<LPX_BF16, STAGED>(layout, ntmax)
                                 : pick<LPX_BF16X3, STAGED>(layout, ntmax);
}

}  // namespace batchk

}  // namespace lpx

using namespace lpx;
using namespace lpx::batchk;

struct lpx_batch {
    int32_t n = 0;
    int precision = 0, layout = 0, ntmax = 2;
    std::vector<int32_t> K, Np;
    std::vector<int64_t> E;
    std::vector<int32_t> order;       // instance index of each table slot
    Item* host_items = nullptr;       // pinned host copy of the table
    Item* dev_items = nullptr;
    unsigned long long* counter = nullptr;
    unsigned char* darr = nullptr;    // every instance's D in MFMA operand order
    std::vector<int64_t> darr_off;    // byte offset of each slot's arrangement
    int64_t darr_bytes = 0;
    int64_t total_tiles = 0, lds = 0;
    int grid = 0;
    bool staged = false;  // staged kernel (32-element tiles) or direct kernel (16)
    int tile_e = 16;
    int ldu = 0, ldo = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t copied = nullptr;      // the table copy of the last submit is done
    int device = -1;
};

namespace {

lpx_status hip_err(hipError_t e, const char* what) {
    return set_error(LPX_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

void free_batch(lpx_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->copied) (void)hipEventDestroy(b->copied);
    if (b->dev_items) (void)hipFree(b->dev_items);
    if (b->counter) (void)hipFree(b->counter);
    if (b->darr) (void)hipFree(b->darr);
    if (b->host_items) (void)hipHostFree(b->host_items);
    delete b;
}

// Fills the pinned table from the descriptors (shapes already validated).
lpx_status fill_table(lpx_batch* b, const lpx_contract_desc* items, const lpx_record* recs) {
    int64_t tile = 0;
    b->lds = b->staged ? 4 * (int64_t)b->ldu * 4 + 2 * (int64_t)b->ldo * 4 : 0;
    for (int32_t slot = 0; slot < b->n; ++slot) {
        const int32_t i = b->order[slot];
        const lpx_contract_desc& c = items[i];
        lpx_record r = recs ? recs[i] : default_record(b->precision);
        lpx_record r0 = r;
        r0.prefetch = 0;  // geometry without LDS staging; the D bit is decided below
        ContractGeom g;
        lpx_status s = contract_geometry(c.K, c.Np, c.E, c.layout, r0, &g);
        if (s != LPX_OK) return s;
        Item& it = b->host_items[slot];
        std::memset(&it, 0, sizeof it);
        it.a.D = c.D;
        it.a.u = c.u;
        it.a.out = c.out;
        it.a.E = c.E;
        it.a.ntiles = ceil_div(c.E, b->tile_e);
        it.a.K = c.K;
        it.a.Np = c.Np;
        it.a.nt = g.nt;
        it.a.nrb = g.nrb;
        it.a.np_div = make_divider(c.Np);
        it.a.nsteps = g.nsteps;
        it.a.ldu = g.ldu;
        it.a.ldo = g.ldo;
        it.a.np_vec = (c.Np % 4) == 0;
        it.a.e_vec = (c.E % 4) == 0;
        it.a.stream_out = (int64_t)c.K * c.E * c.Np * 4 >= ((int64_t)32 << 20);
        it.tile_begin = tile;
        const int64_t frag_bytes = b->precision == LPX_FP32 ? 4 : (b->precision == LPX_BF16 ? 16 : 32);
        const int64_t dbytes = g.nfrag * frag_bytes;
        b->darr_off.push_back(b->darr_bytes);
        b->darr_bytes += round_up(dbytes, 256);
        // direct kernel: D staged in LDS when the record keeps D on chip
        // (LDS or registers); the staged kernel reads D from global memory
        it.d_lds = !b->staged && (r.prefetch & 5) != 0 && dbytes <= kLdsBudget;
        if (it.d_lds) b->lds = std::max(b->lds, dbytes);
        tile += it.a.ntiles;
    }
    b->total_tiles = tile;
    return LPX_OK;
}

lpx_status check_items(const lpx_contract_desc* items, const lpx_record* recs, int32_t n,
                       int* precision, int* layout, int* ntmax) {
    if (!items || n <= 0) return set_error(LPX_ERR_INVALID_ARG, "need n > 0 descriptors");
    *precision = recs ? recs[0].precision : LPX_FP32;
    *layout = items[0].layout;
    *ntmax = 2;
    for (int32_t i = 0; i < n; ++i) {
        // The batch stages D only when it fits its own budget, so the
        // record is checked with LDS staging off.
        lpx_record rr = recs ? recs[i] : default_record(LPX_FP32);
        rr.prefetch = 0;
        const lpx_record* r = &rr;
        ContractGeom g;
        lpx_status s = validate_contract(&items[i], r, &g);
        if (s != LPX_OK) {
            std::string why = last_error_text();  // set_error overwrites it
            return set_error(s, "instance %d: %s", i, why.c_str());
        }
        if ((r ? r->precision : LPX_FP32) != *precision || items[i].layout != *layout)
            return set_error(LPX_ERR_UNSUPPORTED,
                             "instance %d: a batch needs one precision and one layout", i);
        if (items[i].K == 0 || items[i].Np == 0 || items[i].E == 0)
            return set_error(LPX_ERR_INVALID_ARG, "instance %d has a zero size", i);
        *ntmax = std::max(*ntmax, g.ntmax);
    }
    return LPX_OK;
}

lpx_status create(const lpx_contract_desc* items, const lpx_record* recs, int32_t n,
                  lpx_batch** out) {
    int precision, layout, ntmax;
    lpx_status s = check_items(items, recs, n, &precision, &layout, &ntmax);
    if (s != LPX_OK) return s;
    lpx_batch* b = new lpx_batch;
    b->n = n;
    b->precision = precision;
    b->layout = layout;
    b->ntmax = ntmax;
    for (int32_t i = 0; i < n; ++i) {
        b->K.push_back(items[i].K);
        b->Np.push_back(items[i].Np);
        b->E.push_back(items[i].E);
    }
    // Staged kernel when its rings fit in LDS for every instance.
    {
        int64_t ldu = 0, ldo = 0;
        lpx_record rs = default_record(precision);
        rs.tile_e = kTileS;
        rs.prefetch = kPfS;
        bool fits = true;
        for (int32_t i = 0; i < n && fits; ++i) {
            ContractGeom g;
            lpx_problem p{items[i].K, items[i].Np, items[i].E, layout, precision};
            (void)p;
            if (contract_geometry(items[i].K, items[i].Np, items[i].E, layout, rs, &g) != LPX_OK) {
                fits = false;
                break;
            }
            // the batch kernel is compiled for the batch's largest i-block
            // count: its loader rounds set the u slot size
            const ContractShape cs = contract_shape(kTileS, ntmax, kPfS);
            const int64_t rounds = 256LL * cs.nlw * loader_per_lane(kTileS, ntmax, cs.nlw);
            ldu = std::max({ldu, (int64_t)g.ldu, rounds});
            ldo = std::max(ldo, (int64_t)g.ldo);
        }
        clear_error();
        b->staged = fits && 4 * ldu * 4 + 2 * ldo * 4 <= kMaxLdsPerWorkgroup;
        b->tile_e = b->staged ? kTileS : 16;
        b->ldu = (int)ldu;
        b->ldo = (int)ldo;
    }
    b->order.resize(n);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int32_t x, int32_t y) {
        auto cost = [&](int32_t i) { return (double)items[i].K * items[i].Np * items[i].Np * items[i].E; };
        return cost(x) > cost(y);
    });
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->host_items, sizeof(Item) * n, hipHostMallocDefault);
    if (e != hipSuccess) { free_batch(b); return hip_err(e, "batch host table"); }
    if ((s = fill_table(b, items, recs)) != LPX_OK) { free_batch(b); return s; }
    if ((e = hipMalloc((void**)&b->dev_items, sizeof(Item) * n)) != hipSuccess ||
        (e = hipMalloc((void**)&b->darr, (size_t)b->darr_bytes)) != hipSuccess ||
        (e = hipMalloc((void**)&b->counter, sizeof(unsigned long long))) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
        free_batch(b);
        return hip_err(e, "batch allocation");
    }
    BatchFn fn = b->staged ? pick_any<true>(precision, layout, ntmax)
                           : pick_any<false>(precision, layout, ntmax);
    const int threads = b->staged ? contract_shape(kTileS, ntmax, kPfS).threads : kThreadsB;
    DeviceInfo dev;
    if ((s = current_device_info(&dev)) != LPX_OK) { free_batch(b); return s; }
    if (b->lds > 64 * 1024) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds);
        if (e != hipSuccess) { free_batch(b); return hip_err(e, "batch LDS attribute"); }
    }
    int nb = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fn),
                                                     threads, (size_t)b->lds);
    if (e != hipSuccess) { free_batch(b); return hip_err(e, "batch occupancy"); }
    if (nb <= 0) { free_batch(b); return set_error(LPX_ERR_UNSUPPORTED, "batch kernel cannot be resident"); }
    int64_t grid = (int64_t)nb * dev.num_cu;
    const int64_t need = b->staged ? b->total_tiles : ceil_div(b->total_tiles, kChunk);
    b->grid = (int)std::max<int64_t>(1, std::min(grid, need));

    for (int32_t slot = 0; slot < n; ++slot) b->host_items[slot].a.Darr = b->darr + b->darr_off[slot];

    // Capture the launches once: the D arrangement, then the direct kernel
    // after its counter reset or the staged kernel.
    BatchArgs args{b->dev_items, b->counter, b->total_tiles, n, b->ldu, b->ldo};
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const dim3 ag(kern::kArrangeBlocks, (unsigned)std::min(n, 65535)), ab(kern::kArrangeThreads);
        if (precision == LPX_FP32)
            hipLaunchKernelGGL(arrange_all<LPX_FP32>, ag, ab, 0, b->cap_stream, b->dev_items, n);
        else if (precision == LPX_BF16)
            hipLaunchKernelGGL(arrange_all<LPX_BF16>, ag, ab, 0, b->cap_stream, b->dev_items, n);
        else
            hipLaunchKernelGGL(arrange_all<LPX_BF16X3>, ag, ab, 0, b->cap_stream, b->dev_items, n);
        if (!b->staged)
            hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, b->cap_stream, b->counter);
        void* kargs[] = {&args};
        hipError_t le = hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3(b->grid),
                                        dim3(threads), kargs, (size_t)b->lds, b->cap_stream);
        e = hipStreamEndCapture(b->cap_stream, &b->graph);
        if (e == hipSuccess && le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { free_batch(b); return hip_err(e, "batch graph capture"); }
    *out = b;
    return LPX_OK;
}

lpx_status replay(lpx_batch* b, void* stream) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(b->dev_items, b->host_items, sizeof(Item) * b->n,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(b->copied, st);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, st);
    if (e != hipSuccess) return hip_err(e, "batch replay");
    return LPX_OK;
}

}  // namespace

extern "C" {

lpx_status lpx_batch_submit(const lpx_contract_desc* items, const lpx_record* recs, int32_t n,
                            lpx_batch** h, void* stream) {
    clear_error();
    try {
        if (!h) return set_error(LPX_ERR_INVALID_ARG, "handle pointer is NULL");
        if (*h == nullptr) {
            // Records: the caller's, else the tuning cache's, else the default.
            std::vector<lpx_record> rv;
            if (!recs && items && n > 0) {
                rv.resize(n);
                for (int32_t i = 0; i < n; ++i) {
                    lpx_problem p{items[i].K, items[i].Np, items[i].E, items[i].layout, LPX_FP32};
                    if (tuned_lookup(p, &rv[i]) != LPX_OK) rv[i] = default_record(LPX_FP32);
                }
                clear_error();
                recs = rv.data();
            }
            lpx_batch* b = nullptr;
            lpx_status s = create(items, recs, n, &b);
            if (s != LPX_OK) return s;
            s = replay(b, stream);
            if (s != LPX_OK) { free_batch(b); return s; }
            *h = b;
            return LPX_OK;
        }
        lpx_batch* b = *h;
        if (!items || n != b->n)
            return set_error(LPX_ERR_INVALID_ARG, "update needs the batch's %d descriptors", b->n);
        for (int32_t i = 0; i < n; ++i) {
            if (items[i].K != b->K[i] || items[i].Np != b->Np[i] || items[i].E != b->E[i] ||
                items[i].layout != b->layout)
                return set_error(LPX_ERR_INVALID_ARG, "instance %d changed shape; create a new batch", i);
            lpx_record r = default_record(b->precision);
            ContractGeom g;
            lpx_status s = validate_contract(&items[i], &r, &g);
            if (s != LPX_OK) {
                std::string why = last_error_text();
                return set_error(s, "instance %d: %s", i, why.c_str());
            }
        }
        // The previous table copy must have finished before it is rewritten.
        hipError_t e = hipEventSynchronize(b->copied);
        if (e != hipSuccess) return hip_err(e, "batch update");
        for (int32_t slot = 0; slot < b->n; ++slot) {
            const lpx_contract_desc& c = items[b->order[slot]];
            b->host_items[slot].a.D = c.D;
            b->host_items[slot].a.u = c.u;
            b->host_items[slot].a.out = c.out;
        }
        return replay(b, stream);
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_batch_info(const lpx_batch* b, int64_t* total_tiles, int32_t* tile_e,
                          int32_t* grid, int64_t* lds_bytes) {
    clear_error();
    if (!b) return set_error(LPX_ERR_INVALID_ARG, "batch is NULL");
    if (total_tiles) *total_tiles = b->total_tiles;
    if (tile_e) *tile_e = b->tile_e;
    if (grid) *grid = b->grid;
    if (lds_bytes) *lds_bytes = b->lds;
    return LPX_OK;
}

lpx_status lpx_batch_destroy(lpx_batch* b) {
    clear_error();
    free_batch(b);
    return LPX_OK;
}

}  // extern "C"
