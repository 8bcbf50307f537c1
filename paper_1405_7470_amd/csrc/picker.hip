// Variant selection: features, the picker model file, lpx_pick_variant.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "lpx_internal.h"

namespace lpx {

lpx_status launch_mlp_pick(const float* P, const float* feats, int ncand, const float* mean,
                           const float* stdv, float* pred, int* best, void* stream);

namespace {

constexpr char kMagic[8] = {'L', 'P', 'X', 'P', 'I', 'C', 'K', '1'};
constexpr uint32_t kVersion = 1;
constexpr int kMaxCand = LPX_MAX_RECORDS;

uint32_t fnv1a(const unsigned char* p, size_t n) {
    uint32_t h = 2166136261u;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 16777619u;
    }
    return h;
}

struct Header {
    char magic[8];
    uint32_t version, nfeat, hidden, nparams;
};

}  // namespace

lpx_status features(const lpx_problem& p, const lpx_record& r, float* f) {
    ContractGeom g;
    lpx_status s = contract_geometry(p.K, p.Np, p.E, p.layout, r, &g);
    if (s != LPX_OK && s != LPX_ERR_UNSUPPORTED) return s;
    const double rows16 = 16.0 * ceil_div((int64_t)p.K * p.Np, 16);  // stacked row blocks
    f[0] = (float)std::log2((double)p.Np);
    f[1] = (float)std::log2((double)p.E);
    f[2] = (float)p.K;
    f[3] = (float)p.layout;
    f[4] = (float)std::log2((double)r.tile_e);
    f[5] = (float)((r.prefetch & 4) ? 2 : (r.prefetch & 1));  // D: global, LDS, registers
    f[6] = (float)(((r.prefetch >> 1) & 1) + ((r.prefetch >> 3) & 1));  // u, u + output staged
    f[7] = (float)std::log2((double)r.unroll);
    f[8] = (float)r.precision;
    f[9] = (float)((rows16 - (double)p.K * p.Np) / rows16);
    // 16-byte alignment of rows (Np % 4 == 0) and of element runs
    // (E % 4 == 0): they switch the kernels between vector and scalar
    // accesses, which log2 Np and log2 E cannot express
    f[10] = (float)(2 * (p.Np % 4 == 0) + (p.E % 4 == 0));
    f[11] = (float)((double)g.lds_bytes / (double)kMaxLdsPerWorkgroup);
    f[12] = (float)r.order;  // element tiles over the grid: cyclic or blocked
    return LPX_OK;
}

}  // namespace lpx

using namespace lpx;

struct lpx_picker {
    float mean[LPX_MLP_FEATURES], stdv[LPX_MLP_FEATURES];
    std::vector<float> params;  // host copy
    int device = -1;
    float* d_params = nullptr;  // device: params, mean, std, feats, pred
    float* d_mean = nullptr;
    float* d_std = nullptr;
    float* d_feats = nullptr;
    float* d_pred = nullptr;
    int* d_best = nullptr;
    std::mutex mu;
    std::map<std::tuple<int, int, int64_t, int, int>, lpx_record> cache;
};

namespace {

void free_picker(lpx_picker* m) {
    if (!m) return;
    for (void* p : {(void*)m->d_params, (void*)m->d_mean, (void*)m->d_std, (void*)m->d_feats,
                    (void*)m->d_pred, (void*)m->d_best})
        if (p) (void)hipFree(p);
    delete m;
}

lpx_status model_err(const char* path, const char* why) {
    return set_error(LPX_ERR_MODEL, "picker model %s: %s", path, why);
}

}  // namespace

extern "C" {

lpx_status lpx_features(const lpx_problem* p, const lpx_record* r, float* out) {
    clear_error();
    if (!p || !out) return set_error(LPX_ERR_INVALID_ARG, "NULL pointer");
    lpx_status s = check_record(r);
    if (s != LPX_OK) return s;
    if (p->K <= 0 || p->Np <= 0 || p->E <= 0 || p->Np > kMaxNp)
        return set_error(LPX_ERR_INVALID_ARG, "features need 0 < K, 0 < Np <= 128, 0 < E");
    return features(*p, *r, out);
}

lpx_status lpx_picker_save(const char* path, const float* params, const float* mean,
                           const float* stdv) {
    clear_error();
    if (!path || !params || !mean || !stdv) return set_error(LPX_ERR_INVALID_ARG, "NULL pointer");
    std::vector<unsigned char> buf(sizeof(Header));
    Header h;
    std::memcpy(h.magic, kMagic, 8);
    h.version = kVersion;
    h.nfeat = LPX_MLP_FEATURES;
    h.hidden = LPX_MLP_HIDDEN;
    h.nparams = LPX_MLP_PARAMS;
    std::memcpy(buf.data(), &h, sizeof h);
    auto put = [&](const float* v, size_t n) {
        const unsigned char* b = reinterpret_cast<const unsigned char*>(v);
        buf.insert(buf.end(), b, b + n * sizeof(float));
    };
    put(mean, LPX_MLP_FEATURES);
    put(stdv, LPX_MLP_FEATURES);
    put(params, LPX_MLP_PARAMS);
    const uint32_t sum = fnv1a(buf.data(), buf.size());
    const unsigned char* sb = reinterpret_cast<const unsigned char*>(&sum);
    buf.insert(buf.end(), sb, sb + 4);
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(LPX_ERR_INVALID_ARG, "cannot open %s for writing", path);
    const size_t w = std::fwrite(buf.data(), 1, buf.size(), f);
    const int c = std::fclose(f);
    if (w != buf.size() || c != 0) return set_error(LPX_ERR_INTERNAL, "short write to %s", path);
    return LPX_OK;
}

lpx_status lpx_picker_load(const char* path, lpx_picker** out) {
    clear_error();
    try {
        if (!path || !out) return set_error(LPX_ERR_INVALID_ARG, "NULL pointer");
        *out = nullptr;
        FILE* f = std::fopen(path, "rb");
        if (!f) return model_err(path, "cannot be opened");
        std::vector<unsigned char> buf;
        unsigned char tmp[4096];
        size_t r;
        while ((r = std::fread(tmp, 1, sizeof tmp, f)) > 0) buf.insert(buf.end(), tmp, tmp + r);
        std::fclose(f);
        const size_t want = sizeof(Header) +
                            (2 * LPX_MLP_FEATURES + LPX_MLP_PARAMS) * sizeof(float) + 4;
        if (buf.size() != want) return model_err(path, "wrong size");
        Header h;
        std::memcpy(&h, buf.data(), sizeof h);
        if (std::memcmp(h.magic, kMagic, 8) != 0) return model_err(path, "bad magic");
        if (h.version != kVersion) return model_err(path, "unsupported version");
        if (h.nfeat != LPX_MLP_FEATURES || h.hidden != LPX_MLP_HIDDEN ||
            h.nparams != LPX_MLP_PARAMS)
            return model_err(path, "network dimensions differ");
        uint32_t sum;
        std::memcpy(&sum, buf.data() + want - 4, 4);
        if (sum != fnv1a(buf.data(), want - 4)) return model_err(path, "checksum mismatch");
        lpx_picker* m = new lpx_picker;
        const float* v = reinterpret_cast<const float*>(buf.data() + sizeof(Header));
        std::memcpy(m->mean, v, sizeof m->mean);
        std::memcpy(m->stdv, v + LPX_MLP_FEATURES, sizeof m->stdv);
        m->params.assign(v + 2 * LPX_MLP_FEATURES, v + 2 * LPX_MLP_FEATURES + LPX_MLP_PARAMS);
        for (int i = 0; i < LPX_MLP_FEATURES; ++i)
            if (!std::isfinite(m->mean[i]) || !std::isfinite(m->stdv[i]) || m->stdv[i] < 0.f) {
                free_picker(m);
                return model_err(path, "non-finite or negative standardisation");
            }
        for (float x : m->params)
            if (!std::isfinite(x)) {
                free_picker(m);
                return model_err(path, "non-finite weights");
            }
        *out = m;
        return LPX_OK;
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_picker_params(const lpx_picker* m, float* params, float* mean, float* stdv) {
    clear_error();
    if (!m) return set_error(LPX_ERR_INVALID_ARG, "picker is NULL");
    if (params) std::memcpy(params, m->params.data(), LPX_MLP_PARAMS * sizeof(float));
    if (mean) std::memcpy(mean, m->mean, sizeof m->mean);
    if (stdv) std::memcpy(stdv, m->stdv, sizeof m->stdv);
    return LPX_OK;
}

lpx_status lpx_picker_free(lpx_picker* m) {
    clear_error();
    free_picker(m);
    return LPX_OK;
}

lpx_status lpx_pick_variant(const lpx_problem* p, int32_t mode, lpx_picker* model,
                            void* stream, lpx_record* out) {
    clear_error();
    try {
        if (!p || !out) return set_error(LPX_ERR_INVALID_ARG, "NULL pointer");
        if (p->precision < LPX_FP32 || p->precision > LPX_BF16X3)
            return set_error(LPX_ERR_INVALID_ARG, "unknown precision %d", p->precision);
        if (p->K < 0 || p->Np < 0 || p->E < 0 || p->Np > kMaxNp ||
            (p->layout != LPX_ELEMENT_MAJOR && p->layout != LPX_DOF_MAJOR))
            return set_error(LPX_ERR_INVALID_ARG, "bad problem");
        if (mode == LPX_PICK_UNTUNED) {
            *out = default_record(p->precision);
            return LPX_OK;
        }
        if (mode == LPX_PICK_EXHAUSTIVE) return tuned_lookup(*p, out);
        if (mode != LPX_PICK_LEARNED) return set_error(LPX_ERR_INVALID_ARG, "unknown mode %d", mode);
        if (!model) return set_error(LPX_ERR_MODEL, "LEARNED needs a loaded picker model");
        if (p->K == 0 || p->Np == 0 || p->E == 0) {
            *out = default_record(p->precision);
            return LPX_OK;
        }
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return set_error(LPX_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
        std::lock_guard<std::mutex> lock(model->mu);
        auto key = std::make_tuple(p->K, p->Np, p->E, p->layout, p->precision);
        auto it = model->cache.find(key);
        if (it != model->cache.end() && model->device == dev) {
            *out = it->second;
            return LPX_OK;
        }
        if (model->device != dev) {  // (re)upload the weights to this device
            for (void* q : {(void*)model->d_params, (void*)model->d_mean, (void*)model->d_std,
                            (void*)model->d_feats, (void*)model->d_pred, (void*)model->d_best})
                if (q) (void)hipFree(q);
            model->d_params = model->d_mean = model->d_std = model->d_feats = model->d_pred = nullptr;
            model->d_best = nullptr;
            model->cache.clear();
            if ((e = hipMalloc((void**)&model->d_params, LPX_MLP_PARAMS * 4)) != hipSuccess ||
                (e = hipMalloc((void**)&model->d_mean, LPX_MLP_FEATURES * 4)) != hipSuccess ||
                (e = hipMalloc((void**)&model->d_std, LPX_MLP_FEATURES * 4)) != hipSuccess ||
                (e = hipMalloc((void**)&model->d_feats, kMaxCand * LPX_MLP_FEATURES * 4)) != hipSuccess ||
                (e = hipMalloc((void**)&model->d_pred, kMaxCand * 4)) != hipSuccess ||
                (e = hipMalloc((void**)&model->d_best, 4)) != hipSuccess ||
                (e = hipMemcpy(model->d_params, model->params.data(), LPX_MLP_PARAMS * 4,
                               hipMemcpyHostToDevice)) != hipSuccess ||
                (e = hipMemcpy(model->d_mean, model->mean, sizeof model->mean,
                               hipMemcpyHostToDevice)) != hipSuccess ||
                (e = hipMemcpy(model->d_std, model->stdv, sizeof model->stdv,
                               hipMemcpyHostToDevice)) != hipSuccess)
                return set_error(LPX_ERR_HIP, "picker upload: %s", hipGetErrorString(e));
            model->device = dev;
        }
        // Candidates that the kernels support for this shape.
        lpx_record all[kMaxCand];
        int32_t nall = 0;
        lpx_status s = lpx_record_enumerate(p, all, kMaxCand, &nall);
        if (s != LPX_OK) return s;
        std::vector<lpx_record> cand;
        std::vector<float> feats;
        for (int32_t i = 0; i < nall && i < kMaxCand; ++i) {
            ContractGeom g;
            if (contract_geometry(p->K, p->Np, p->E, p->layout, all[i], &g) != LPX_OK) continue;
            float f[LPX_MLP_FEATURES];
            if ((s = features(*p, all[i], f)) != LPX_OK) return s;
            cand.push_back(all[i]);
            feats.insert(feats.end(), f, f + LPX_MLP_FEATURES);
        }
        clear_error();
        if (cand.empty()) return set_error(LPX_ERR_UNSUPPORTED, "no candidate record fits");
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        int best = -1;
        if ((e = hipMemcpyAsync(model->d_feats, feats.data(), feats.size() * 4,
                                hipMemcpyHostToDevice, st)) != hipSuccess)
            return set_error(LPX_ERR_HIP, "picker features: %s", hipGetErrorString(e));
        s = launch_mlp_pick(model->d_params, model->d_feats, (int)cand.size(), model->d_mean,
                            model->d_std, model->d_pred, model->d_best, stream);
        if (s != LPX_OK) return s;
        if ((e = hipMemcpyAsync(&best, model->d_best, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return set_error(LPX_ERR_HIP, "picker result: %s", hipGetErrorString(e));
        if (best < 0 || best >= (int)cand.size())
            return set_error(LPX_ERR_INTERNAL, "picker returned index %d", best);
        *out = cand[best];
        model->cache[key] = cand[best];
        return LPX_OK;
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

}  // extern "C"
