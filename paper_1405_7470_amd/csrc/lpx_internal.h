// Internal declarations shared by the liblpx translation units.
#pragma once

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/lpx.h"

namespace lpx {

// gfx950 limits used by host-side validation (no HIP call needed).
constexpr int64_t kMaxLdsPerWorkgroup = 160 * 1024;
constexpr int kMaxNp = 128;

// Thread-local last-error text; set_error returns its status so call sites
// can `return set_error(...)`.
lpx_status set_error(lpx_status s, const char* fmt, ...)
    __attribute__((format(printf, 2, 3)));
void clear_error();
const char* last_error_text();

// Record defaults and checks.
lpx_record default_record(int precision);
lpx_status check_record(const lpx_record* rec);

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Work-group shape of a contraction kernel instance (host and device agree
// on it through this one function).  Without a staged u tile (prefetch bit
// 1 clear): four waves per 16-element block, splitting its (k, i-block)
// pairs.  With one: min(4 * tile_e/16, 8) compute waves (4 when D is in
// registers and tile_e = 64), four per block, each taking bpw = 4 * nb /
// ncw blocks of every tile (two or four at tile_e = 64, so a wave does more
// MFMA work per work-group barrier); nlw
// loader waves (1, or tile_e * ntmax / 128 when larger, so that a loader
// wave loads at most 8 16-byte chunks per lane and tile); and with a staged
// output tile (bit 3) four store waves: the write-back is three quarters
// of the traffic and needs that many waves issuing stores to keep HBM busy.
struct ContractShape {
    int ncw, wpe, bpw, nlw, nsw, threads;
};
constexpr ContractShape contract_shape(int tile_e, int ntmax, int prefetch) {
    const bool pf_u = (prefetch & 2) != 0;
    const bool pf_o = (prefetch & 8) != 0;
    const int nb = tile_e / 16;
    // D in registers at tile_e = 64: one compute wave per SIMD taking all
    // four blocks of its part (its registers allow reading the next block's
    // operands during the current block's MFMAs)
    const int ncw_cap = (prefetch & 4) && tile_e == 64 ? 4 : 8;
    const int ncw = pf_u ? (4 * nb < ncw_cap ? 4 * nb : ncw_cap) : 4 * nb;
    const int nlw = pf_u ? (tile_e * ntmax / 128 > 1 ? tile_e * ntmax / 128 : 1) : 0;
    const int nsw = pf_o ? 4 : 0;
    return ContractShape{ncw, 4, 4 * nb / ncw, nlw, nsw, 64 * (ncw + nlw + nsw)};
}
// 16-byte chunks one loader wave loads per u tile (nlw loader waves; a
// tile holds at most tile_e * 16 * ntmax floats).
constexpr int loader_per_lane(int tile_e, int ntmax, int nlw) {
    return (tile_e * 16 * ntmax / 4 + 64 * nlw - 1) / (64 * nlw);
}
inline int64_t ceil_div(int64_t x, int64_t m) { return (x + m - 1) / m; }

// Exact n / d for 0 <= n < 2^31 and 1 <= d <= 2^16 as one 32x32-bit
// multiply and a shift (division by an invariant integer, Granlund and
// Montgomery 1994): with l = ceil(log2 d) and m = ceil(2^(31+l) / d), the
// error of n*m / 2^(31+l) against n/d stays below 2^-l <= 1/d, so the floor
// is exact.
struct Divider {
    uint32_t m;
    int sh;
};
inline Divider make_divider(int d) {
    int l = 0;
    while ((1 << l) < d) ++l;
    Divider v;
    v.m = (uint32_t)(((1ULL << (31 + l)) + (uint64_t)d - 1) / (uint64_t)d);
    v.sh = 31 + l;
    return v;
}

// Geometry of one contraction launch, derived from (problem, record) on the
// host.  Every quantity the kernel's indexing assumes is computed here.
struct ContractGeom {
    int prec = 0, layout = 0;
    int tile_e = 16, prefetch = 0, unroll = 1;
    int order = 0;     // element tiles over the grid: 0 cyclic, 1 blocked
    int threads = 256;  // work-group size: 4 wave64s per 16 elements of the tile
    int kstep = 4;     // reduction length of one MFMA (4 fp32, 32 bf16)
    int nt = 0;        // i-blocks of 16 rows: ceil(Np / 16)
    int ntmax = 2;     // compiled bound on nt: 2, 4 or 8
    int nsteps = 0;    // MFMA k-steps: ceil(Np / kstep)
    int nrb = 0;       // stacked row blocks of 16 rows of D as [K*Np][Np]: ceil(K*Np / 16)
    int ldu = 0;       // LDS ring slot stride of a staged u tile (floats)
    int ldo = 0;       // LDS ring slot stride of a staged output tile (floats)
    int dg = 0;        // dG volume term: the metric epilogue in the store waves
    int ldo_g = 0;     // dg: float offset of the geometric factors in an output slot
    int64_t ntiles = 0;
    int64_t nfrag = 0;     // staged D fragments: nrb*nsteps*64 lanes
    int64_t lds_bytes = 0; // dynamic LDS per work-group (0 if no prefetch)
};

// Fills g; returns LPX_OK or LPX_ERR_UNSUPPORTED (with error text) when the
// shape is outside what the record's kernels are built for.
// dg: geometry of the dG volume kernels (the output slots also carry the
// tile's geometric factors).
lpx_status contract_geometry(int K, int Np, int64_t E, int layout,
                             const lpx_record& r, ContractGeom* g, bool dg = false);

// Every check of lpx_contract / lpx_gemm that needs no HIP call.
lpx_status validate_contract(const lpx_contract_desc* c, const lpx_record* rec, ContractGeom* g,
                             bool dg = false);
// The dG volume term: every check without a HIP call; *chosen receives the
// record used (rec, or the default NULL stands for).
lpx_status validate_dg(const lpx_dg_volume_desc* c, const lpx_record* rec, ContractGeom* g,
                       lpx_record* chosen);
lpx_status validate_gemm(const lpx_gemm_desc* g, const lpx_record* rec, bool* noop);
bool overlaps(const void* a, int64_t abytes, const void* b, int64_t bbytes);
bool mul_overflows(int64_t a, int64_t b, int64_t* r);
bool aligned16(const void* p);

// Tuning cache (per device): lookup returns LPX_ERR_NOT_TUNED on a miss.
lpx_status tuned_lookup(const lpx_problem& p, lpx_record* out);
lpx_status tuned_store(const lpx_problem& p, const lpx_record& r);

// Stream-ordered workspace of `bytes` on `stream` from the library's own
// memory pool of the current device (freed with hipFreeAsync on the same
// stream; freed blocks stay in the pool for reuse).
lpx_status workspace_alloc(void** p, size_t bytes, void* stream, const char* what);

// Launches the contraction kernel for a validated problem.

// noalloc: D's arrangement (if the record reads D from memory) goes to the
// library's static device scratch instead of a per-call workspace; the
// caller has checked darr_bytes(g) against LPX_NOALLOC_SCRATCH_BYTES.
lpx_status launch_contract(const lpx_contract_desc& c, const ContractGeom& g,
                           void* stream, bool noalloc = false, const float* G = nullptr);

// Bytes of D's MFMA-order arrangement in memory for a geometry (0 when the
// record keeps D in LDS or registers).
int64_t darr_bytes(const ContractGeom& g);

// GEMM tiling of a record (defaults filled in); LPX_ERR_UNSUPPORTED if that
// tiling is not built for the record's precision.
lpx_status gemm_tiles(const lpx_record& r, int* tm, int* tn, int* tk);
lpx_status launch_gemm(const lpx_gemm_desc& d, const lpx_record& r, void* stream);

// Elementwise bf16 split kernel launch (n > 0, pointers validated).
lpx_status launch_split_bf16(const float* x, uint16_t* hi, uint16_t* lo,
                             int64_t n, void* stream);

// The 12 cost-model features of (problem, record) into f[12].
lpx_status features(const lpx_problem& p, const lpx_record& r, float* f);

// Device properties of the current device, cached per device.
struct DeviceInfo {
    int device = -1;
    int num_cu = 0;
    int max_lds_per_block = 0;
};
lpx_status current_device_info(DeviceInfo* out);

}  // namespace lpx
