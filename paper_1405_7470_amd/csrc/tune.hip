// Exhaustive autotuner, tuning cache and variant selection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "lpx_internal.h"

namespace lpx {
namespace {

using TuneKey = std::tuple<int, int, int, int64_t, int, int>;  // dev,K,Np,E,layout,prec

std::mutex g_mu;
std::map<TuneKey, lpx_record> g_tuned;

lpx_status key_for(const lpx_problem& p, TuneKey* k) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(LPX_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    *k = TuneKey(dev, p.K, p.Np, p.E, p.layout, p.precision);
    return LPX_OK;
}

// Overwrites the flush buffer: the caches then hold its dirty lines and
// none of the tuned problem's, so the timed launch also pays for writing
// back what it evicts, as it does when it follows other work.
__global__ void flush_kernel(float4* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

lpx_status tuned_lookup(const lpx_problem& p, lpx_record* out) {
    TuneKey k;
    lpx_status s = key_for(p, &k);
    if (s != LPX_OK) return s;
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_tuned.find(k);
    if (it == g_tuned.end())
        return set_error(LPX_ERR_NOT_TUNED, "no tuning result for K=%d Np=%d E=%lld", p.K, p.Np,
                         (long long)p.E);
    *out = it->second;
    return LPX_OK;
}

lpx_status tuned_store(const lpx_problem& p, const lpx_record& r) {
    TuneKey k;
    lpx_status s = key_for(p, &k);
    if (s != LPX_OK) return s;
    std::lock_guard<std::mutex> lock(g_mu);
    g_tuned[k] = r;
    return LPX_OK;
}

}  // namespace lpx

using namespace lpx;

extern "C" {

lpx_status lpx_autotune(const lpx_contract_desc* c, int32_t precision, int32_t warmup,
                        int32_t reps, void* flush, int64_t flush_bytes, void* stream,
                        lpx_record* best, float* times_us, int32_t cap, int32_t* n) {
    clear_error();
    try {
        if (!c || !best) return set_error(LPX_ERR_INVALID_ARG, "descriptor or best is NULL");
        if (warmup < 0 || reps < 1 || cap < 0 || (cap > 0 && !times_us))
            return set_error(LPX_ERR_INVALID_ARG, "bad warmup/reps/times array");
        if (precision < LPX_FP32 || precision > LPX_BF16X3)
            return set_error(LPX_ERR_INVALID_ARG, "unknown precision %d", precision);
        if (flush && (flush_bytes <= 0 || flush_bytes % 16 ||
                      (reinterpret_cast<uintptr_t>(flush) & 15)))
            return set_error(LPX_ERR_INVALID_ARG, "flush buffer must be 16-byte aligned and sized");
        lpx_record def = default_record(precision);
        lpx_status s = lpx_contract_validate(c, &def);
        if (s != LPX_OK) return s;
        lpx_problem p{c->K, c->Np, c->E, c->layout, precision};
        lpx_record recs[LPX_MAX_RECORDS];
        int32_t nrec = 0;
        s = lpx_record_enumerate(&p, recs, LPX_MAX_RECORDS, &nrec);
        if (s != LPX_OK) return s;
        if (n) *n = nrec;
        std::vector<float> med(nrec, INFINITY);
        if (c->K == 0 || c->Np == 0 || c->E == 0) {
            *best = def;
        } else {
            Events ev;
            hipError_t e = hipEventCreate(&ev.a);
            if (e == hipSuccess) e = hipEventCreate(&ev.b);
            if (e != hipSuccess)
                return set_error(LPX_ERR_HIP, "hipEventCreate: %s", hipGetErrorString(e));
            hipStream_t st = reinterpret_cast<hipStream_t>(stream);
            std::vector<float> t(reps);
            for (int32_t r = 0; r < nrec; ++r) {
                if (lpx_contract_validate(c, &recs[r]) != LPX_OK) continue;  // e.g. LDS
                for (int32_t w = 0; w < warmup; ++w)
                    if ((s = lpx_contract(c, &recs[r], stream)) != LPX_OK) return s;
                for (int32_t q = 0; q < reps; ++q) {
                    if (flush) {
                        hipLaunchKernelGGL(flush_kernel, dim3(2048), dim3(256), 0, st,
                                           reinterpret_cast<float4*>(flush), flush_bytes / 16);
                        if ((e = hipGetLastError()) != hipSuccess) break;
                    }
                    if ((e = hipEventRecord(ev.a, st)) != hipSuccess) break;
                    if ((s = lpx_contract(c, &recs[r], stream)) != LPX_OK) return s;
                    if ((e = hipEventRecord(ev.b, st)) != hipSuccess) break;
                    if ((e = hipEventSynchronize(ev.b)) != hipSuccess) break;
                    float ms = 0.f;
                    if ((e = hipEventElapsedTime(&ms, ev.a, ev.b)) != hipSuccess) break;
                    t[q] = ms * 1000.f;
                }
                if (e != hipSuccess)
                    return set_error(LPX_ERR_HIP, "timing: %s", hipGetErrorString(e));
                std::sort(t.begin(), t.end());
                med[r] = t[reps / 2];
            }
            int32_t arg = -1;
            for (int32_t r = 0; r < nrec; ++r)
                if (std::isfinite(med[r]) && (arg < 0 || med[r] < med[arg])) arg = r;
            if (arg < 0) return set_error(LPX_ERR_UNSUPPORTED, "no candidate record ran");
            *best = recs[arg];
            if ((s = tuned_store(p, recs[arg])) != LPX_OK) return s;
        }
        for (int32_t r = 0; r < std::min(cap, nrec); ++r) times_us[r] = med[r];
        return LPX_OK;
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_tune_cache_insert(const lpx_problem* p, const lpx_record* rec) {
    clear_error();
    if (!p) return set_error(LPX_ERR_INVALID_ARG, "problem is NULL");
    lpx_status s = check_record(rec);
    if (s != LPX_OK) return s;
    if (rec->precision != p->precision)
        return set_error(LPX_ERR_INVALID_ARG, "record precision differs from the problem's");
    return tuned_store(*p, *rec);
}

lpx_status lpx_tune_cache_clear(void) {
    clear_error();
    std::lock_guard<std::mutex> lock(g_mu);
    g_tuned.clear();
    return LPX_OK;
}

}  // extern "C"
