// Host side of the C ABI: validation, records, error reporting, dispatch.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstring>
#include <mutex>
#include <vector>

#include "lpx_internal.h"

namespace lpx {

namespace {
thread_local char g_last_error[512] = "";
}

lpx_status set_error(lpx_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return s;
}

void clear_error() { g_last_error[0] = '\0'; }

const char* last_error_text() { return g_last_error; }

lpx_record default_record(int precision) {
    lpx_record r;
    std::memset(&r, 0, sizeof r);
    r.version = LPX_RECORD_VERSION;
    r.precision = (uint8_t)precision;
    r.tile_e = 16;
    r.prefetch = 0;
    r.unroll = 1;
    return r;
}

// The prefetch bit sets of sec. 2.4.4 that are built: bits 0 (D in LDS)
// and 2 (D in registers) exclude each other, and bit 3 (staged output)
// needs bit 1 (staged u, the pipeline its store waves join).
static const uint8_t kPrefetchSets[] = {0, 1, 2, 3, 4, 6, 10, 11, 14};

static bool prefetch_valid(unsigned pf) {
    for (uint8_t v : kPrefetchSets)
        if (v == pf) return true;
    return false;
}

lpx_status check_record(const lpx_record* rec) {
    if (!rec) return set_error(LPX_ERR_INVALID_ARG, "record is NULL");
    if (rec->version != LPX_RECORD_VERSION)
        return set_error(LPX_ERR_INVALID_ARG, "record version %u, expected %u",
                         rec->version, LPX_RECORD_VERSION);
    if (rec->precision > LPX_BF16X3)
        return set_error(LPX_ERR_INVALID_ARG, "unknown precision %u", rec->precision);
    if (rec->tile_e != 16 && rec->tile_e != 32 && rec->tile_e != 64)
        return set_error(LPX_ERR_INVALID_ARG, "tile_e %u not in {16,32,64}", rec->tile_e);
    if (!prefetch_valid(rec->prefetch))
        return set_error(LPX_ERR_INVALID_ARG, "prefetch %u not in {0,1,2,3,4,6,10,11,14}",
                         rec->prefetch);
    if (rec->unroll != 1 && rec->unroll != 2 && rec->unroll != 4)
        return set_error(LPX_ERR_INVALID_ARG, "unroll %u not in {1,2,4}", rec->unroll);
    if (rec->assume_tile_divides > 1)
        return set_error(LPX_ERR_INVALID_ARG, "assume_tile_divides %u not in {0,1}",
                         rec->assume_tile_divides);
    if (rec->order > 1) return set_error(LPX_ERR_INVALID_ARG, "order %u not in {0,1}", rec->order);
    for (uint8_t b : rec->reserved0)
        if (b) return set_error(LPX_ERR_INVALID_ARG, "reserved record bytes must be 0");
    if (rec->reserved1) return set_error(LPX_ERR_INVALID_ARG, "reserved record bytes must be 0");
    return LPX_OK;
}

lpx_status contract_geometry(int K, int Np, int64_t E, int layout,
                             const lpx_record& r, ContractGeom* g, bool dg) {
    g->dg = dg ? 1 : 0;
    g->prec = r.precision;
    g->layout = layout;
    g->tile_e = r.tile_e;
    g->prefetch = r.prefetch;
    g->unroll = r.unroll;
    g->order = r.order;
    g->kstep = (r.precision == LPX_FP32) ? 4 : 32;
    g->nt = (int)ceil_div(Np, 16);
    g->ntmax = g->nt <= 2 ? 2 : (g->nt <= 4 ? 4 : 8);
    g->threads = contract_shape(r.tile_e, g->ntmax, r.prefetch).threads;
    g->nsteps = (int)ceil_div(Np, g->kstep);
    g->ntiles = ceil_div(E, r.tile_e);
    if ((int64_t)K * Np > (int64_t)INT32_MAX - 16)
        return set_error(LPX_ERR_UNSUPPORTED, "K*Np = %lld stacked operator rows exceed 2^31 - 16",
                         (long long)K * Np);
    g->nrb = (int)ceil_div((int64_t)K * Np, 16);
    g->nfrag = (int64_t)g->nrb * g->nsteps * 64;
    // D's MFMA-order arrangement (in LDS or global memory) is indexed by
    // fragment with 32-bit integers, the bf16x3 lo plane after the hi plane.
    {
        const int64_t planes = r.precision == LPX_BF16X3 ? 2 : 1;
        if (g->nfrag * planes > (int64_t)INT32_MAX)
            return set_error(LPX_ERR_UNSUPPORTED,
                             "K=%d Np=%d needs %lld D fragments per plane; the operator "
                             "arrangement holds at most 2^31 - 1 (over all planes)",
                             K, Np, (long long)g->nfrag);
    }
    // A staged u tile is a raw copy of the tile (tile_e * Np floats) plus
    // slack for reads of padding columns up to the next multiple of 32.
    // u ring slot stride in floats: a raw tile copy with slack for reads of
    // padding columns (up to the next multiple of 32), and room for every
    // chunk the loader waves write (tiles are loaded in whole rounds of
    // 64 chunks per loader wave).
    {
        const ContractShape cs = contract_shape(r.tile_e, g->ntmax, r.prefetch);
        const int nlw = cs.nlw > 0 ? cs.nlw : 1;
        const int64_t need = (int64_t)r.tile_e * round_up(Np, 32) + 32;
        const int64_t rounds = 256LL * nlw * loader_per_lane(r.tile_e, g->ntmax, nlw);
        g->ldu = (int)(need > rounds ? need : rounds);
    }
    // A staged output tile: element-major K*tile_e*Np floats, DOF-major
    // K*Np rows of tile_e + 4 floats (both multiples of 4 floats).
    // The dG volume kernels append the tile's geometric factors (tile_e*K*K
    // floats) to each output slot.
    const int64_t ldo_out = layout == LPX_ELEMENT_MAJOR
                                ? round_up((int64_t)K * r.tile_e * Np, 4)
                                : (int64_t)K * Np * (r.tile_e + 4);
    const int64_t ldo = ldo_out + (dg ? round_up((int64_t)r.tile_e * K * K, 4) : 0);
    g->ldo = (r.prefetch & 8) && ldo <= kMaxLdsPerWorkgroup ? (int)ldo : 0;
    g->ldo_g = dg && g->ldo ? (int)ldo_out : 0;
    if (r.prefetch & 4) {
        // D in registers: each wave holds the fragments of its row blocks,
        // which needs Np <= 64, four waves per 16-element block and all of
        // the row blocks in one chunk.
        const ContractShape cs = contract_shape(r.tile_e, g->ntmax, r.prefetch);
        const int pmax = (3 * g->ntmax + cs.wpe - 1) / cs.wpe;
        if (g->ntmax > 4 || cs.wpe != 4 || g->nrb > cs.wpe * pmax)
            return set_error(LPX_ERR_UNSUPPORTED,
                             "prefetch=%u (D in registers) needs Np <= 64 and ceil(K*Np/16) <= %d "
                             "(K=%d Np=%d)",
                             r.prefetch, cs.wpe * pmax, K, Np);
    }
    g->lds_bytes = 0;
    if (r.prefetch) {
        const int64_t frag_bytes =
            r.precision == LPX_FP32 ? 4 : (r.precision == LPX_BF16 ? 16 : 32);
        const int64_t ring_bytes = 4 * (int64_t)g->ldu * 4;  // four slots
        g->lds_bytes = ((r.prefetch & 1) ? g->nfrag * frag_bytes : 0) +
                       ((r.prefetch & 2) ? ring_bytes : 0) +
                       ((r.prefetch & 8) ? 2 * ldo * 4 : 0);
        if (g->lds_bytes > kMaxLdsPerWorkgroup)
            return set_error(LPX_ERR_UNSUPPORTED,
                             "prefetch=%u needs %lld bytes of LDS per work-group for K=%d "
                             "Np=%d (limit %lld)",
                             r.prefetch, (long long)g->lds_bytes, K, Np,
                             (long long)kMaxLdsPerWorkgroup);
    }
    return LPX_OK;
}

lpx_status current_device_info(DeviceInfo* out) {
    static std::mutex mu;
    static std::vector<DeviceInfo> cache;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return set_error(LPX_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1);
    DeviceInfo& d = cache[dev];
    if (d.device < 0) {
        int ncu = 0, lds = 0;
        e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess)
            return set_error(LPX_ERR_HIP, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
        d.device = dev;
        d.num_cu = ncu;
        d.max_lds_per_block = lds;
    }
    *out = d;
    return LPX_OK;
}

}  // namespace lpx

using namespace lpx;

namespace lpx {

bool overlaps(const void* a, int64_t abytes, const void* b, int64_t bbytes) {
    auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return abytes > 0 && bbytes > 0 && pa < pb + (uintptr_t)bbytes &&
           pb < pa + (uintptr_t)abytes;
}

bool mul_overflows(int64_t a, int64_t b, int64_t* r) {
    return __builtin_mul_overflow(a, b, r);
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Every check of lpx_contract that needs no HIP call.  On LPX_OK, g holds
// the launch geometry; g->ntiles == 0 marks a zero-size no-op.
lpx_status validate_contract(const lpx_contract_desc* c, const lpx_record* rec,
                             ContractGeom* g, bool dg) {
    g->ntiles = 0;
    if (!c) return set_error(LPX_ERR_INVALID_ARG, "descriptor is NULL");
    lpx_record r = rec ? *rec : default_record(LPX_FP32);
    lpx_status s = check_record(&r);
    if (s != LPX_OK) return s;
    if (c->K < 0 || c->Np < 0 || c->E < 0)
        return set_error(LPX_ERR_INVALID_ARG, "negative size K=%d Np=%d E=%lld", c->K, c->Np,
                         (long long)c->E);
    if (c->layout != LPX_ELEMENT_MAJOR && c->layout != LPX_DOF_MAJOR)
        return set_error(LPX_ERR_INVALID_ARG, "unknown layout %d", c->layout);
    if (c->reserved != 0) return set_error(LPX_ERR_INVALID_ARG, "reserved must be 0");
    int64_t uelems, oelems, delems;
    if (mul_overflows(c->E, c->Np, &uelems) || mul_overflows(uelems, c->K, &oelems) ||
        mul_overflows((int64_t)c->Np * c->Np, c->K, &delems) || oelems > INT64_MAX / 4)
        return set_error(LPX_ERR_INVALID_ARG, "size product overflows int64");
    if (c->Np > kMaxNp)
        return set_error(LPX_ERR_UNSUPPORTED, "Np=%d above the supported %d", c->Np, kMaxNp);
    if (r.assume_tile_divides && c->E % r.tile_e != 0)
        return set_error(LPX_ERR_ASSUMPTION, "record assumes E %% %u == 0 but E = %lld",
                         r.tile_e, (long long)c->E);
    if (c->K == 0 || c->Np == 0 || c->E == 0) return LPX_OK;  // zero-trip loop
    if (!c->D || !c->u || !c->out) return set_error(LPX_ERR_INVALID_ARG, "NULL D, u or out");
    if (!aligned16(c->D) || !aligned16(c->u) || !aligned16(c->out))
        return set_error(LPX_ERR_INVALID_ARG, "D, u and out must be 16-byte aligned");
    if (overlaps(c->out, oelems * 4, c->u, uelems * 4) ||
        overlaps(c->out, oelems * 4, c->D, delems * 4))
        return set_error(LPX_ERR_ALIAS, "out overlaps D or u");
    return contract_geometry(c->K, c->Np, c->E, c->layout, r, g, dg);
}

lpx_status validate_dg(const lpx_dg_volume_desc* c, const lpx_record* rec, ContractGeom* g,
                       lpx_record* chosen) {
    g->ntiles = 0;
    if (!c) return set_error(LPX_ERR_INVALID_ARG, "descriptor is NULL");
    if (c->K > LPX_DG_MAX_K)
        return set_error(LPX_ERR_UNSUPPORTED, "dG volume term with K=%d above %d", c->K,
                         LPX_DG_MAX_K);
    lpx_contract_desc cd;
    cd.K = c->K;
    cd.Np = c->Np;
    cd.E = c->E;
    cd.layout = c->layout;
    cd.reserved = c->reserved;
    cd.D = c->D;
    cd.u = c->u;
    cd.out = c->out;
    lpx_record r;
    lpx_status s;
    if (rec) {
        r = *rec;
        if ((s = check_record(&r)) != LPX_OK) return s;
        if (!(r.prefetch & 8))
            return set_error(LPX_ERR_UNSUPPORTED,
                             "the dG volume term needs a staged output tile (prefetch 10, 11 or "
                             "14), got prefetch %u", r.prefetch);
        s = validate_contract(&cd, &r, g, true);
    } else {
        // the first of these that fits the shape
        static const uint8_t kDefaults[4][2] = {{64, 14}, {64, 10}, {32, 10}, {16, 10}};
        s = LPX_ERR_UNSUPPORTED;
        for (const auto& d : kDefaults) {
            r = default_record(LPX_FP32);
            r.tile_e = d[0];
            r.prefetch = d[1];
            s = validate_contract(&cd, &r, g, true);
            if (s != LPX_ERR_UNSUPPORTED) break;
        }
    }
    if (chosen) *chosen = r;
    if (s != LPX_OK || g->ntiles == 0) return s;
    if (!c->G) return set_error(LPX_ERR_INVALID_ARG, "NULL G");
    if (!aligned16(c->G)) return set_error(LPX_ERR_INVALID_ARG, "G must be 16-byte aligned");
    const int64_t gbytes = c->E * c->K * c->K * 4, obytes = c->E * c->K * c->Np * 4;
    if (overlaps(c->out, obytes, c->G, gbytes))
        return set_error(LPX_ERR_ALIAS, "out overlaps G");
    return LPX_OK;
}


lpx_status validate_gemm(const lpx_gemm_desc* g, const lpx_record* rec, bool* noop) {
    *noop = true;
    if (!g) return set_error(LPX_ERR_INVALID_ARG, "descriptor is NULL");
    lpx_record r = rec ? *rec : default_record(LPX_FP32);
    lpx_status s = check_record(&r);
    if (s != LPX_OK) return s;
    if (g->M < 0 || g->N < 0 || g->K < 0)
        return set_error(LPX_ERR_INVALID_ARG, "negative size");
    int tm, tn, tk;
    s = gemm_tiles(r, &tm, &tn, &tk);
    if (s != LPX_OK) return s;
    if (g->M == 0 || g->N == 0) return LPX_OK;  // nothing to write
    if (!g->A && g->K > 0) return set_error(LPX_ERR_INVALID_ARG, "NULL A");
    if (!g->B && g->K > 0) return set_error(LPX_ERR_INVALID_ARG, "NULL B");
    if (!g->C) return set_error(LPX_ERR_INVALID_ARG, "NULL C");
    if (g->lda < g->K || g->ldb < g->N || g->ldc < g->N)
        return set_error(LPX_ERR_INVALID_ARG, "leading dimension below the row length");
    if ((g->K > 0 && (!aligned16(g->A) || !aligned16(g->B))) || !aligned16(g->C))
        return set_error(LPX_ERR_INVALID_ARG, "A, B and C must be 16-byte aligned");
    int64_t abytes, bbytes, cbytes;
    if (mul_overflows(g->M, g->lda, &abytes) || mul_overflows(g->K, g->ldb, &bbytes) ||
        mul_overflows(g->M, g->ldc, &cbytes) || abytes > INT64_MAX / 4 ||
        bbytes > INT64_MAX / 4 || cbytes > INT64_MAX / 4)
        return set_error(LPX_ERR_INVALID_ARG, "size product overflows int64");
    if (overlaps(g->C, cbytes * 4, g->A, abytes * 4) || overlaps(g->C, cbytes * 4, g->B, bbytes * 4))
        return set_error(LPX_ERR_ALIAS, "C overlaps A or B");
    *noop = false;
    return LPX_OK;
}

}  // namespace lpx

extern "C" {

const char* lpx_version(void) { return "lpx 0.1.0 gfx950"; }

const char* lpx_status_string(lpx_status s) {
    switch (s) {
        case LPX_OK: return "LPX_OK";
        case LPX_ERR_INVALID_ARG: return "LPX_ERR_INVALID_ARG";
        case LPX_ERR_UNSUPPORTED: return "LPX_ERR_UNSUPPORTED";
        case LPX_ERR_ASSUMPTION: return "LPX_ERR_ASSUMPTION";
        case LPX_ERR_ALIAS: return "LPX_ERR_ALIAS";
        case LPX_ERR_HIP: return "LPX_ERR_HIP";
        case LPX_ERR_MODEL: return "LPX_ERR_MODEL";
        case LPX_ERR_NOT_TUNED: return "LPX_ERR_NOT_TUNED";
        case LPX_ERR_INTERNAL: return "LPX_ERR_INTERNAL";
        default: return "LPX_ERR_UNKNOWN";
    }
}

const char* lpx_last_error(void) { return last_error_text(); }

lpx_status lpx_record_default(int32_t precision, lpx_record* out) {
    clear_error();
    if (!out) return set_error(LPX_ERR_INVALID_ARG, "out is NULL");
    if (precision < LPX_FP32 || precision > LPX_BF16X3)
        return set_error(LPX_ERR_INVALID_ARG, "unknown precision %d", precision);
    *out = default_record(precision);
    return LPX_OK;
}

lpx_status lpx_record_validate(const lpx_record* rec) {
    clear_error();
    return check_record(rec);
}

lpx_status lpx_record_describe(const lpx_record* rec, char* buf, size_t len) {
    clear_error();
    if (!buf || len == 0) return set_error(LPX_ERR_INVALID_ARG, "buffer is NULL or empty");
    lpx_status s = check_record(rec);
    if (s != LPX_OK) {
        buf[0] = '\0';
        return s;
    }
    static const char* prec[] = {"fp32", "bf16", "bf16x3"};
    snprintf(buf, len, "%s tile_e=%u prefetch=%u unroll=%u%s%s gemm=%ux%ux%u",
             prec[rec->precision], rec->tile_e, rec->prefetch, rec->unroll,
             rec->order ? " order=blocked" : "",
             rec->assume_tile_divides ? " assume(E%tile_e==0)" : "", rec->gemm_tm,
             rec->gemm_tn, rec->gemm_tk);
    return LPX_OK;
}

lpx_status lpx_record_enumerate(const lpx_problem* p, lpx_record* recs, int32_t cap,
                                int32_t* n) {
    clear_error();
    if (!p || !n) return set_error(LPX_ERR_INVALID_ARG, "problem or n is NULL");
    if (cap < 0 || (cap > 0 && !recs))
        return set_error(LPX_ERR_INVALID_ARG, "bad output array (cap %d)", cap);
    if (p->precision < LPX_FP32 || p->precision > LPX_BF16X3)
        return set_error(LPX_ERR_INVALID_ARG, "unknown precision %d", p->precision);
    static const uint8_t tiles[] = {16, 32, 64};
    static const uint8_t unrolls[] = {1, 2, 4};
    int32_t count = 0;
    for (uint8_t ord = 0; ord < 2; ++ord)
        for (uint8_t t : tiles)
            for (uint8_t pf : kPrefetchSets)
                for (uint8_t un : unrolls) {
                    if (count < cap) {
                        lpx_record r = default_record(p->precision);
                        r.tile_e = t;
                        r.prefetch = pf;
                        r.unroll = un;
                        r.order = ord;
                        recs[count] = r;
                    }
                    ++count;
                }
    *n = count;
    return LPX_OK;
}

lpx_status lpx_contract_lds_bytes(const lpx_problem* p, const lpx_record* rec,
                                  int64_t* bytes) {
    clear_error();
    if (!p || !bytes) return set_error(LPX_ERR_INVALID_ARG, "problem or bytes is NULL");
    lpx_status s = check_record(rec);
    if (s != LPX_OK) return s;
    if (p->K < 0 || p->Np < 0 || p->E < 0)
        return set_error(LPX_ERR_INVALID_ARG, "negative size");
    if (p->Np > kMaxNp)
        return set_error(LPX_ERR_UNSUPPORTED, "Np=%d above %d", p->Np, kMaxNp);
    ContractGeom g;
    s = contract_geometry(p->K, p->Np, p->E, p->layout, *rec, &g);
    *bytes = g.lds_bytes;
    return s;
}

lpx_status lpx_contract_validate(const lpx_contract_desc* c, const lpx_record* rec) {
    clear_error();
    try {
        ContractGeom g;
        return validate_contract(c, rec, &g);
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_contract(const lpx_contract_desc* c, const lpx_record* rec, void* stream) {
    clear_error();
    try {
        ContractGeom g;
        lpx_status s = validate_contract(c, rec, &g);
        if (s != LPX_OK || g.ntiles == 0) return s;
        return launch_contract(*c, g, stream);
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_contract_noalloc(const lpx_contract_desc* c, const lpx_record* rec,
                                void* stream) {
    clear_error();
    try {
        ContractGeom g;
        lpx_status s = validate_contract(c, rec, &g);
        if (s != LPX_OK || g.ntiles == 0) return s;
        if (darr_bytes(g) > LPX_NOALLOC_SCRATCH_BYTES)
            return set_error(LPX_ERR_UNSUPPORTED,
                             "lpx_contract_noalloc: D's arrangement needs %lld bytes, above the "
                             "%d-byte scratch (K=%d Np=%d)",
                             (long long)darr_bytes(g), LPX_NOALLOC_SCRATCH_BYTES, c->K, c->Np);
        return launch_contract(*c, g, stream, true);
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_dg_volume_validate(const lpx_dg_volume_desc* c, const lpx_record* rec,
                                  lpx_record* chosen) {
    clear_error();
    try {
        ContractGeom g;
        lpx_record r;
        lpx_status s = validate_dg(c, rec, &g, &r);
        if (chosen) *chosen = r;
        return s;
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_dg_volume(const lpx_dg_volume_desc* c, const lpx_record* rec, void* stream) {
    clear_error();
    try {
        ContractGeom g;
        lpx_record r;
        lpx_status s = validate_dg(c, rec, &g, &r);
        if (s != LPX_OK || g.ntiles == 0) return s;
        lpx_contract_desc cd;
        cd.K = c->K;
        cd.Np = c->Np;
        cd.E = c->E;
        cd.layout = c->layout;
        cd.reserved = 0;
        cd.D = c->D;
        cd.u = c->u;
        cd.out = c->out;
        return launch_contract(cd, g, stream, false, c->G);
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_gemm_validate(const lpx_gemm_desc* g, const lpx_record* rec) {
    clear_error();
    try {
        bool noop;
        return validate_gemm(g, rec, &noop);
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_gemm(const lpx_gemm_desc* g, const lpx_record* rec, void* stream) {
    clear_error();
    try {
        bool noop;
        lpx_status s = validate_gemm(g, rec, &noop);
        if (s != LPX_OK || noop) return s;
        return launch_gemm(*g, rec ? *rec : default_record(LPX_FP32), stream);
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

lpx_status lpx_split_bf16(const float* x, uint16_t* hi, uint16_t* lo, int64_t n,
                          void* stream) {
    clear_error();
    try {
        if (n < 0) return set_error(LPX_ERR_INVALID_ARG, "negative n");
        if (n == 0) return LPX_OK;
        if (!x || !hi || !lo) return set_error(LPX_ERR_INVALID_ARG, "NULL pointer");
        if ((reinterpret_cast<uintptr_t>(x) & 3u) || (reinterpret_cast<uintptr_t>(hi) & 1u) ||
            (reinterpret_cast<uintptr_t>(lo) & 1u))
            return set_error(LPX_ERR_INVALID_ARG, "misaligned pointer");
        if (n > INT64_MAX / 4) return set_error(LPX_ERR_INVALID_ARG, "n too large");
        if (overlaps(hi, n * 2, x, n * 4) || overlaps(lo, n * 2, x, n * 4) ||
            overlaps(hi, n * 2, lo, n * 2))
            return set_error(LPX_ERR_ALIAS, "hi/lo overlap x or each other");
        return launch_split_bf16(x, hi, lo, n, stream);
    } catch (...) {
        return set_error(LPX_ERR_INTERNAL, "unexpected C++ exception");
    }
}

}  // extern "C"
