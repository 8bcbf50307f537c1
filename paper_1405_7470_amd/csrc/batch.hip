// Ragged batch of contractions in one graph, each instance run by its own
// record's kernel.
//
// Instances are grouped by the kernel their record (and i-block bound)
// selects; each group is one persistent launch of that kernel's batch-run
// twin (contract_runs_kernel), which executes the contraction's own tile
// code on runs of consecutive tiles of one instance at a time.  Every
// instance's tiles are cut into runs of about the same length, and the runs
// are dealt to the group's work-groups largest first, each to the
// work-group with the least work so far (cost of a tile: its row blocks x
// k-steps), so a work-group changes instance -- and stages or loads D again
// -- only between runs.  Records that read D from memory get its MFMA-order
// arrangement from the first graph nodes, into a buffer the batch owns.
//
// The nodes (arrangements, then one launch per group on kBranches parallel
// branches) are captured once into a HIP graph on library-owned streams;
// lpx_batch_submit replays it on the caller's stream after copying the
// (possibly updated) descriptor table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <queue>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "contract_dispatch.h"

namespace lpx {
namespace batchk {

// D of the listed instances in MFMA operand order, written to their slices
// of the batch's arrangement buffer (a.Darr).
template <int PREC>
__global__ __launch_bounds__(kern::kArrangeThreads) void arrange_list(
    const kern::ContractArgs* __restrict__ items, const int32_t* __restrict__ idx, int m) {
    // constant-address-space reads: scalar loads, and the descriptors'
    // pointers are known to point to global memory (see contract_runs_kernel)
    typedef __attribute__((address_space(4))) const kern::ContractArgs CItem;
    typedef __attribute__((address_space(4))) const int32_t CInt;
    const CItem* citems = (const CItem*)items;
    const CInt* cidx = (const CInt*)idx;
    for (int i = blockIdx.y; i < m; i += gridDim.y) {
        const kern::ContractArgs a = kern::load_args(citems + cidx[i]);
        kern::stage_d<PREC, kern::kArrangeThreads * kern::kArrangeBlocks>(
            a, const_cast<unsigned char*>(a.Darr),
            blockIdx.x * kern::kArrangeThreads + threadIdx.x);
    }
}

RunsFn select_runs(const ContractGeom& g) {
    const bool em = g.layout == LPX_ELEMENT_MAJOR;
    const int nt = g.ntmax, t = g.tile_e, pf = g.prefetch, un = g.unroll;
    switch (g.prec) {
        case LPX_FP32:
            return em ? runs_instance<LPX_FP32, LPX_ELEMENT_MAJOR>(nt, t, pf, un)
                      : runs_instance<LPX_FP32, LPX_DOF_MAJOR>(nt, t, pf, un);
        case LPX_BF16:
            return em ? runs_instance<LPX_BF16, LPX_ELEMENT_MAJOR>(nt, t, pf, un)
                      : runs_instance<LPX_BF16, LPX_DOF_MAJOR>(nt, t, pf, un);
        default:
            return em ? runs_instance<LPX_BF16X3, LPX_ELEMENT_MAJOR>(nt, t, pf, un)
                      : runs_instance<LPX_BF16X3, LPX_DOF_MAJOR>(nt, t, pf, un);
    }
}

// One persistent launch: the instances whose records select kernel `fn`.
struct Group {
    RunsFn fn = nullptr;
    int threads = 0;
    int64_t lds = 0;       // largest dynamic LDS of its instances
    int grid = 0;
    int64_t run_off = 0;   // first entry in the batch's run table
    int64_t wg_off = 0;    // first entry in the batch's work-group table
    int64_t tiles = 0;
    std::vector<int32_t> inst;
};

// Runs per work-group in a balanced group: enough to even out the tail,
// few enough that a run is long against its start-up (pipeline fill, D).
constexpr int kRunsPerWg = 3;
constexpr int64_t kMinRunTiles = 4;
// Parallel branches of the graph the group launches are spread over
// (512-instance batch, per-instance learned records, 24 groups: 2 branches
// 4.61 ms, 3 4.04, 4 3.98, 6 4.02, 8 3.94; batch-tuned records, 5 groups:
// 3.54, 3.60, 3.43, 3.55, 3.56 ms).
constexpr int kBranches = 4;

}  // namespace batchk
}  // namespace lpx

using namespace lpx;
using namespace lpx::batchk;

struct lpx_batch {
    int32_t n = 0;
    std::vector<int32_t> K, Np, layout;
    std::vector<int64_t> E;
    std::vector<lpx_record> rec;
    kern::ContractArgs* host_items = nullptr;  // pinned host copy of the table
    kern::ContractArgs* dev_items = nullptr;
    kern::Run* dev_runs = nullptr;
    int32_t* dev_wg = nullptr;
    int32_t* dev_idx = nullptr;      // instances to arrange, per precision
    unsigned char* darr = nullptr;   // D arrangements of the records that read D from memory
    std::vector<Group> groups;
    int64_t arr_off[3] = {0, 0, 0}, arr_cnt[3] = {0, 0, 0};  // FP32, BF16, BF16X3 lists
    int64_t total_tiles = 0, lds_max = 0;
    int grid_total = 0;
    hipStream_t cap_stream = nullptr;
    hipStream_t side[kBranches - 1] = {};  // the graph's other branches during capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t copied = nullptr;     // the table copy of the last submit is done
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
    for (hipStream_t s : b->side)
        if (s) (void)hipStreamDestroy(s);
    if (b->copied) (void)hipEventDestroy(b->copied);
    if (b->dev_items) (void)hipFree(b->dev_items);
    if (b->dev_runs) (void)hipFree(b->dev_runs);
    if (b->dev_wg) (void)hipFree(b->dev_wg);
    if (b->dev_idx) (void)hipFree(b->dev_idx);
    if (b->darr) (void)hipFree(b->darr);
    if (b->host_items) (void)hipHostFree(b->host_items);
    delete b;
}

int prec_slot(int precision) {
    return precision == LPX_FP32 ? 0 : (precision == LPX_BF16 ? 1 : 2);
}

// Every instance checked as lpx_contract checks it, with its own record.
lpx_status check_items(const lpx_contract_desc* items, const lpx_record* recs, int32_t n,
                       std::vector<ContractGeom>* geo) {
    if (!items || n <= 0) return set_error(LPX_ERR_INVALID_ARG, "need n > 0 descriptors");
    geo->resize(n);
    for (int32_t i = 0; i < n; ++i) {
        if (items[i].K == 0 || items[i].Np == 0 || items[i].E == 0)
            return set_error(LPX_ERR_INVALID_ARG, "instance %d has a zero size", i);
        lpx_status s = validate_contract(&items[i], &recs[i], &(*geo)[i]);
        if (s != LPX_OK) {
            std::string why = last_error_text();  // set_error overwrites it
            return set_error(s, "instance %d: %s", i, why.c_str());
        }
    }
    return LPX_OK;
}

// Cuts the group's instances into runs and deals them to at most `gmax`
// work-groups; appends to runs / wg_first (offsets recorded in the group).
void plan_group(Group& G, const std::vector<ContractGeom>& geo, int gmax,
                std::vector<kern::Run>* runs, std::vector<int32_t>* wg_first) {
    int64_t T = 0;
    for (int32_t i : G.inst) T += geo[i].ntiles;
    G.tiles = T;
    const int64_t len = std::max<int64_t>(kMinRunTiles, T / ((int64_t)gmax * kRunsPerWg));
    struct Cut {
        double cost;
        kern::Run run;
    };
    std::vector<Cut> cuts;
    for (int32_t i : G.inst) {
        const int64_t nt = geo[i].ntiles;
        const int64_t nr = (nt + len - 1) / len;
        const double per_tile = (double)geo[i].nrb * geo[i].nsteps;
        for (int64_t r = 0; r < nr; ++r) {
            const int64_t first = nt * r / nr, last = nt * (r + 1) / nr;
            cuts.push_back({per_tile * (double)(last - first),
                            kern::Run{first, i, (int32_t)(last - first)}});
        }
    }
    std::stable_sort(cuts.begin(), cuts.end(),
                     [](const Cut& x, const Cut& y) { return x.cost > y.cost; });
    const int grid = (int)std::min<int64_t>(gmax, (int64_t)cuts.size());
    // least-loaded work-group first (ties: lowest index)
    using Load = std::pair<double, int>;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int w = 0; w < grid; ++w) heap.push({0.0, w});
    std::vector<std::vector<kern::Run>> per(grid);
    for (const Cut& c : cuts) {
        const Load l = heap.top();
        heap.pop();
        per[l.second].push_back(c.run);
        heap.push({l.first + c.cost, l.second});
    }
    G.grid = grid;
    G.run_off = (int64_t)runs->size();
    G.wg_off = (int64_t)wg_first->size();
    int32_t q = 0;
    for (int w = 0; w < grid; ++w) {
        wg_first->push_back(q);
        for (const kern::Run& r : per[w]) runs->push_back(r);
        q += (int32_t)per[w].size();
    }
    wg_first->push_back(q);
}

lpx_status create(const lpx_contract_desc* items, const lpx_record* recs, int32_t n,
                  lpx_batch** out) {
    std::vector<ContractGeom> geo;
    lpx_status s = check_items(items, recs, n, &geo);
    if (s != LPX_OK) return s;
    DeviceInfo dev;
    if ((s = current_device_info(&dev)) != LPX_OK) return s;
    lpx_batch* b = new lpx_batch;
    b->n = n;
    b->device = dev.device;
    for (int32_t i = 0; i < n; ++i) {
        b->K.push_back(items[i].K);
        b->Np.push_back(items[i].Np);
        b->E.push_back(items[i].E);
        b->layout.push_back(items[i].layout);
        b->rec.push_back(recs[i]);
    }
    hipError_t e =
        hipHostMalloc((void**)&b->host_items, sizeof(kern::ContractArgs) * n, hipHostMallocDefault);
    if (e != hipSuccess) { free_batch(b); return hip_err(e, "batch host table"); }

    // kernel per instance, groups, arrangement lists
    std::map<const void*, int> group_of;
    std::vector<int32_t> arr[3];
    std::vector<int64_t> darr_off(n, -1);
    int64_t darr_total = 0;
    for (int32_t i = 0; i < n; ++i) {
        const ContractGeom& g = geo[i];
        if (g.lds_bytes > dev.max_lds_per_block) {
            free_batch(b);
            return set_error(LPX_ERR_UNSUPPORTED, "instance %d needs %lld bytes of LDS", i,
                             (long long)g.lds_bytes);
        }
        RunsFn fn = select_runs(g);
        if (!fn) {
            free_batch(b);
            return set_error(LPX_ERR_INTERNAL, "instance %d: no kernel for a validated record", i);
        }
        auto it = group_of.find(reinterpret_cast<const void*>(fn));
        if (it == group_of.end()) {
            it = group_of.emplace(reinterpret_cast<const void*>(fn), (int)b->groups.size()).first;
            Group G;
            G.fn = fn;
            G.threads = g.threads;
            b->groups.push_back(G);
        }
        Group& G = b->groups[it->second];
        G.inst.push_back(i);
        G.lds = std::max(G.lds, g.lds_bytes);
        b->host_items[i] = contract_args(items[i], g);
        const int64_t db = darr_bytes(g);
        if (db > 0) {
            darr_off[i] = darr_total;
            darr_total += round_up(db, 256);
            arr[prec_slot(g.prec)].push_back(i);
        }
    }
    std::vector<kern::Run> runs;
    std::vector<int32_t> wg_first;
    for (Group& G : b->groups) {
        int nb = 0;
        s = blocks_per_cu(reinterpret_cast<const void*>(G.fn), G.threads, G.lds, dev.device, &nb);
        if (s == LPX_OK && nb <= 0)
            s = set_error(LPX_ERR_UNSUPPORTED, "batch kernel cannot be resident (LDS %lld bytes)",
                          (long long)G.lds);
        if (s != LPX_OK) { free_batch(b); return s; }
        plan_group(G, geo, nb * dev.num_cu, &runs, &wg_first);
        b->total_tiles += G.tiles;
        b->grid_total += G.grid;
        b->lds_max = std::max(b->lds_max, G.lds);
    }
    std::vector<int32_t> idx;
    for (int p = 0; p < 3; ++p) {
        b->arr_off[p] = (int64_t)idx.size();
        b->arr_cnt[p] = (int64_t)arr[p].size();
        idx.insert(idx.end(), arr[p].begin(), arr[p].end());
    }
    if ((e = hipMalloc((void**)&b->dev_items, sizeof(kern::ContractArgs) * n)) != hipSuccess ||
        (e = hipMalloc((void**)&b->dev_runs, sizeof(kern::Run) * runs.size())) != hipSuccess ||
        (e = hipMalloc((void**)&b->dev_wg, sizeof(int32_t) * wg_first.size())) != hipSuccess ||
        (!idx.empty() &&
         (e = hipMalloc((void**)&b->dev_idx, sizeof(int32_t) * idx.size())) != hipSuccess) ||
        (darr_total > 0 && (e = hipMalloc((void**)&b->darr, (size_t)darr_total)) != hipSuccess) ||
        (e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
        free_batch(b);
        return hip_err(e, "batch allocation");
    }
    for (hipStream_t& s : b->side)
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) {
            free_batch(b);
            return hip_err(e, "batch allocation");
        }
    for (int32_t i = 0; i < n; ++i)
        if (darr_off[i] >= 0) b->host_items[i].Darr = b->darr + darr_off[i];
    // the run, work-group and arrangement tables never change: copied once
    if ((e = hipMemcpy(b->dev_runs, runs.data(), sizeof(kern::Run) * runs.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(b->dev_wg, wg_first.data(), sizeof(int32_t) * wg_first.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (!idx.empty() && (e = hipMemcpy(b->dev_idx, idx.data(), sizeof(int32_t) * idx.size(),
                                        hipMemcpyHostToDevice)) != hipSuccess)) {
        free_batch(b);
        return hip_err(e, "batch tables");
    }

    // Capture once: the arrangements, then one launch per group.
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = hipSuccess;
        for (int p = 0; p < 3; ++p) {
            const int m = (int)b->arr_cnt[p];
            if (m == 0) continue;
            const dim3 ag(kern::kArrangeBlocks, (unsigned)std::min(m, 65535)),
                ab(kern::kArrangeThreads);
            const int32_t* list = b->dev_idx + b->arr_off[p];
            if (p == 0)
                hipLaunchKernelGGL(arrange_list<LPX_FP32>, ag, ab, 0, b->cap_stream, b->dev_items,
                                   list, m);
            else if (p == 1)
                hipLaunchKernelGGL(arrange_list<LPX_BF16>, ag, ab, 0, b->cap_stream, b->dev_items,
                                   list, m);
            else
                hipLaunchKernelGGL(arrange_list<LPX_BF16X3>, ag, ab, 0, b->cap_stream,
                                   b->dev_items, list, m);
            if (le == hipSuccess) le = hipGetLastError();
        }
        // The group launches on kBranches branches of the graph (largest
        // groups first, each to the branch with the least work), so that one
        // group's tail overlaps work of the other branches.
        hipStream_t br_stream[kBranches];
        br_stream[0] = b->cap_stream;
        for (int k = 1; k < kBranches; ++k) br_stream[k] = b->side[k - 1];
        hipEvent_t fork = nullptr, join[kBranches] = {};
        if (le == hipSuccess) le = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        for (int k = 1; k < kBranches; ++k)
            if (le == hipSuccess) le = hipEventCreateWithFlags(&join[k], hipEventDisableTiming);
        if (le == hipSuccess) le = hipEventRecord(fork, b->cap_stream);
        for (int k = 1; k < kBranches; ++k)
            if (le == hipSuccess) le = hipStreamWaitEvent(br_stream[k], fork, 0);
        std::vector<std::pair<double, int>> order;  // (-work, group)
        for (int gi = 0; gi < (int)b->groups.size(); ++gi) {
            double w = 0;
            for (int32_t i : b->groups[gi].inst)
                w += (double)geo[i].ntiles * geo[i].tile_e * geo[i].nrb * geo[i].nsteps;
            order.push_back({-w, gi});
        }
        std::sort(order.begin(), order.end());
        double load[kBranches] = {};
        for (const auto& o : order) {
            const Group& G = b->groups[o.second];
            int br = 0;
            for (int k = 1; k < kBranches; ++k)
                if (load[k] < load[br]) br = k;
            load[br] -= o.first;
            kern::RunArgs ra{b->dev_items, b->dev_runs + G.run_off, b->dev_wg + G.wg_off};
            void* kargs[] = {&ra};
            const hipError_t ge = hipLaunchKernel(
                reinterpret_cast<const void*>(G.fn), dim3((unsigned)G.grid), dim3(G.threads),
                kargs, (size_t)G.lds, br_stream[br]);
            if (le == hipSuccess) le = ge;
        }
        for (int k = 1; k < kBranches; ++k) {
            if (le == hipSuccess) le = hipEventRecord(join[k], br_stream[k]);
            if (le == hipSuccess) le = hipStreamWaitEvent(b->cap_stream, join[k], 0);
        }
        e = hipStreamEndCapture(b->cap_stream, &b->graph);
        if (e == hipSuccess && le != hipSuccess) e = le;
        if (fork) (void)hipEventDestroy(fork);
        for (hipEvent_t j : join)
            if (j) (void)hipEventDestroy(j);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { free_batch(b); return hip_err(e, "batch graph capture"); }
    *out = b;
    return LPX_OK;
}

lpx_status replay(lpx_batch* b, void* stream) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(b->dev_items, b->host_items, sizeof(kern::ContractArgs) * b->n,
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
        if (!items) {
            // replay with the table as it is: after its last copy, no host work
            hipStream_t st = reinterpret_cast<hipStream_t>(stream);
            hipError_t e = hipStreamWaitEvent(st, b->copied, 0);
            if (e == hipSuccess) e = hipGraphLaunch(b->exec, st);
            if (e != hipSuccess) return hip_err(e, "batch replay");
            return LPX_OK;
        }
        if (n != b->n)
            return set_error(LPX_ERR_INVALID_ARG, "update needs the batch's %d descriptors", b->n);
        for (int32_t i = 0; i < n; ++i) {
            if (items[i].K != b->K[i] || items[i].Np != b->Np[i] || items[i].E != b->E[i] ||
                items[i].layout != b->layout[i])
                return set_error(LPX_ERR_INVALID_ARG, "instance %d changed shape; create a new batch", i);
            ContractGeom g;
            lpx_status s = validate_contract(&items[i], &b->rec[i], &g);
            if (s != LPX_OK) {
                std::string why = last_error_text();
                return set_error(s, "instance %d: %s", i, why.c_str());
            }
        }
        // The previous table copy must have finished before it is rewritten.
        hipError_t e = hipEventSynchronize(b->copied);
        if (e != hipSuccess) return hip_err(e, "batch update");
        for (int32_t i = 0; i < n; ++i) {
            b->host_items[i].D = items[i].D;
            b->host_items[i].u = items[i].u;
            b->host_items[i].out = items[i].out;
        }
        return replay(b, stream);
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_batch_tune(const lpx_contract_desc* items, int32_t n, int32_t precision,
                          int32_t warmup, int32_t reps, void* stream, lpx_record* recs_out) {
    clear_error();
    try {
        if (!items || n <= 0 || !recs_out)
            return set_error(LPX_ERR_INVALID_ARG, "need n > 0 descriptors and an output array");
        if (warmup < 0 || reps < 1) return set_error(LPX_ERR_INVALID_ARG, "bad warmup/reps");
        if (precision < LPX_FP32 || precision > LPX_BF16X3)
            return set_error(LPX_ERR_INVALID_ARG, "unknown precision %d", precision);
        // groups of instances that share (K, Np, layout)
        std::map<std::tuple<int, int, int>, std::vector<int32_t>> groups;
        for (int32_t i = 0; i < n; ++i) {
            if (items[i].K == 0 || items[i].Np == 0 || items[i].E == 0)
                return set_error(LPX_ERR_INVALID_ARG, "instance %d has a zero size", i);
            lpx_record def = default_record(precision);
            ContractGeom g;
            lpx_status s = validate_contract(&items[i], &def, &g);
            if (s != LPX_OK) {
                std::string why = last_error_text();
                return set_error(s, "instance %d: %s", i, why.c_str());
            }
            groups[std::make_tuple(items[i].K, items[i].Np, items[i].layout)].push_back(i);
        }
        hipEvent_t ea = nullptr, eb = nullptr;
        hipError_t e = hipEventCreate(&ea);
        if (e == hipSuccess) e = hipEventCreate(&eb);
        if (e != hipSuccess) {
            if (ea) (void)hipEventDestroy(ea);
            return hip_err(e, "hipEventCreate");
        }
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        lpx_status status = LPX_OK;
        std::vector<float> t(reps);
        for (auto& kv : groups) {
            const std::vector<int32_t>& idx = kv.second;
            std::vector<lpx_contract_desc> sub;
            for (int32_t i : idx) sub.push_back(items[i]);
            lpx_problem p{items[idx[0]].K, items[idx[0]].Np, items[idx[0]].E,
                          items[idx[0]].layout, precision};
            lpx_record cand[LPX_MAX_RECORDS];
            int32_t ncand = 0;
            if ((status = lpx_record_enumerate(&p, cand, LPX_MAX_RECORDS, &ncand)) != LPX_OK) break;
            float best_t = INFINITY;
            lpx_record best = default_record(precision);
            for (int32_t c = 0; c < ncand && status == LPX_OK; ++c) {
                // the batch lays out its own runs: records that differ only
                // in the tile order run the same code, so one order is timed
                if (cand[c].order != 0) continue;
                std::vector<lpx_record> rv(sub.size(), cand[c]);
                bool fits = true;
                for (const lpx_contract_desc& d : sub) {
                    ContractGeom g;
                    if (validate_contract(&d, &cand[c], &g) != LPX_OK) fits = false;
                }
                clear_error();
                if (!fits) continue;
                lpx_batch* b = nullptr;
                if (create(sub.data(), rv.data(), (int32_t)sub.size(), &b) != LPX_OK) {
                    clear_error();  // e.g. a kernel that cannot be resident
                    continue;
                }
                for (int32_t w = 0; w < warmup && status == LPX_OK; ++w) status = replay(b, stream);
                for (int32_t q = 0; q < reps && status == LPX_OK; ++q) {
                    float ms = 0.f;
                    if ((e = hipEventRecord(ea, st)) == hipSuccess &&
                        (status = replay(b, stream)) == LPX_OK &&
                        (e = hipEventRecord(eb, st)) == hipSuccess &&
                        (e = hipEventSynchronize(eb)) == hipSuccess &&
                        (e = hipEventElapsedTime(&ms, ea, eb)) == hipSuccess)
                        t[q] = ms * 1000.f;
                    if (e != hipSuccess && status == LPX_OK) status = hip_err(e, "batch timing");
                }
                if (status == LPX_OK && (e = hipStreamSynchronize(st)) != hipSuccess)
                    status = hip_err(e, "batch timing");
                free_batch(b);
                if (status != LPX_OK) break;
                std::sort(t.begin(), t.end());
                if (t[reps / 2] < best_t) {
                    best_t = t[reps / 2];
                    best = cand[c];
                }
            }
            if (status != LPX_OK) break;
            for (int32_t i : idx) recs_out[i] = best;
        }
        (void)hipEventDestroy(ea);
        (void)hipEventDestroy(eb);
        return status;
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_batch_info(const lpx_batch* b, int64_t* total_tiles, int32_t* kernels,
                          int32_t* grid, int64_t* lds_bytes) {
    clear_error();
    if (!b) return set_error(LPX_ERR_INVALID_ARG, "batch is NULL");
    if (total_tiles) *total_tiles = b->total_tiles;
    if (kernels) *kernels = (int32_t)b->groups.size();
    if (grid) *grid = b->grid_total;
    if (lds_bytes) *lds_bytes = b->lds_max;
    return LPX_OK;
}

lpx_status lpx_batch_destroy(lpx_batch* b) {
    clear_error();
    free_batch(b);
    return LPX_OK;
}

}  // extern "C"
