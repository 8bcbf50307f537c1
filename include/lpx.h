/*
 * lpx.h -- C ABI of liblpx: code variants of the batched dense contraction
 *
 *     out[k,e,i] = sum_j D[k][i][j] * u[e][j]
 *
 * and of its degenerate case, dense GEMM, on AMD Instinct MI355X (gfx950).
 *
 * Background (Klöckner, "Loo.py: transformation-based code generation for
 * GPUs and CPUs", ARRAY'14):
 *   - the computation is a reduction in the paper's sense (sec. 2.1,
 *     sum(j, D[k,i,j]*u[e,j])); Table 1's "dG FEM volume" and "sgemm" rows
 *     are the workloads it stands for;
 *   - the paper's point is that the instructions, the loop bounds and the
 *     explicitly invoked transformations together fix the generated code
 *     (sec. 1).  Here the transformations are an explicit, immutable value,
 *     the transformation record (lpx_record), passed with every call; each
 *     legal record selects one precompiled gfx950 kernel instance;
 *   - size parameters are plain arguments, as the paper's kernel
 *     parameters are (sec. 2.1), and every call is enqueued on a stream and
 *     returns before the work finishes, as a kernel call on an OpenCL queue
 *     does (sec. 2.2);
 *   - kernels are compiled ahead of time and callable from any host program
 *     (sec. 1): this header has no dependency beyond <stdint.h>/<stddef.h>.
 *
 * Conventions for every entry point:
 *   - Pointers named as "device" are HIP device pointers (global memory of
 *     the current device); "host" pointers are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - The caller owns every buffer it passes and keeps it alive until the
 *     stream has passed the enqueued work.
 *   - Arguments are validated before any HIP call; on error nothing is
 *     enqueued, no output is written, and lpx_last_error() describes the
 *     failure.  No function aborts or throws.
 *   - A problem with a zero size (K, Np or E equal to 0) is a successful
 *     no-op, like a loop whose upper bound lies below its lower bound
 *     (sec. 2.2's generated loop runs zero times for n = 0).
 */
#ifndef LPX_H
#define LPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef int32_t lpx_status;
#define LPX_OK 0
#define LPX_ERR_INVALID_ARG 1 /* NULL/misaligned pointer, negative or     */
                              /* overflowing size, malformed record       */
#define LPX_ERR_UNSUPPORTED 2 /* legal record not built for this shape    */
                              /* (e.g. LDS staging does not fit, Np > 128) */
#define LPX_ERR_ASSUMPTION 3  /* a record's assumption is false for shape */
#define LPX_ERR_ALIAS 4       /* output overlaps an input                 */
#define LPX_ERR_HIP 5         /* HIP runtime/launch error (text kept)     */
#define LPX_ERR_MODEL 6       /* picker model missing/corrupt/version     */
#define LPX_ERR_NOT_TUNED 7   /* no tuning result cached for the shape    */
#define LPX_ERR_INTERNAL 8

/* ------------------------------------------------------------- enums */
/* Arithmetic of the products (a semantics-changing choice the caller opts
 * into; the paper leaves such choices to the user, sec. 1). Accumulation is
 * always FP32.
 *   FP32   : FP32 operands, FP32 MFMA.
 *   BF16   : operands rounded to bfloat16 (nearest-even), BF16 MFMA.
 *   BF16X3 : x = hi + lo with hi = bf16(x), lo = bf16(x - hi); each product
 *            as hi*hi + hi*lo + lo*hi (lo*lo dropped), BF16 MFMA.        */
#define LPX_FP32 0
#define LPX_BF16 1
#define LPX_BF16X3 2

/* Storage of u and out (sec. 2.4.3, array-axis implementation tags; the
 * structure-of-arrays / array-of-structures switch):
 *   ELEMENT_MAJOR: u[e*Np + j],  out[(k*E + e)*Np + i]
 *   DOF_MAJOR    : u[j*E + e],   out[(k*Np + i)*E + e]
 * D is always D[(k*Np + i)*Np + j].                                     */
#define LPX_ELEMENT_MAJOR 0
#define LPX_DOF_MAJOR 1

/* ------------------------------------------------ transformation record */
#define LPX_RECORD_VERSION 1u

/* One code variant.  Every field is one transformation of sec. 2.4:
 *   tile_e   : split_iname(e, tile_e) with the outer index mapped to the
 *              work-group grid axis (sec. 2.4.1 eq. (1), sec. 2.4.2);
 *              16, 32 or 64 elements per work-group tile.  Inside a tile,
 *              e is split again by 16 (the MFMA column block) and i by 16
 *              (the MFMA row block); each 16-element block has four wave64s
 *              that split its (k, i-block) pairs (with a staged u tile,
 *              at most eight compute waves per work-group, each taking
 *              tile_e / 32 blocks of a 64-element tile).
 *   prefetch : storage of the operands (add_prefetch / precompute, sec.
 *              2.4.4), a bit set from {0,1,2,3,4,6,10,11,14}:
 *              bit 0: all of D is staged in LDS once per work-group, in
 *              MFMA operand order and converted to the operand precision;
 *              bit 1: each u tile is staged in LDS by dedicated loader waves
 *              that keep three tiles in flight (a four-slot LDS ring, one
 *              work-group barrier per tile);
 *              bit 2: D is precomputed into private memory -- each wave
 *              keeps the D fragments of its own 16-row blocks of the
 *              stacked operators in registers for the whole kernel
 *              (Np <= 64 and ceil(K*Np/16) <= 12, else LPX_ERR_UNSUPPORTED; unroll does not apply, the
 *              k-step loop is fully unrolled);
 *              bit 3 (needs bit 1): each output tile is staged in LDS and
 *              written back by dedicated store waves with contiguous
 *              16-byte stores one tile behind the compute waves, which then
 *              touch no global memory at all.
 *              Bits 0 and 2 are exclusive.  A clear bit means that array's
 *              MFMA operands are loaded from global memory straight into
 *              registers (or, for the output, stored straight from them);
 *              with bits 0 and 2 both clear, D is read from an MFMA-order
 *              copy that a pre-pass kernel writes once per call into a
 *              stream-ordered workspace (nrb*nsteps*64 fragments; taken
 *              from and returned to a memory pool the library creates and
 *              owns per device -- the device's default pool is not
 *              touched).  The untuned default record is such a record: it
 *              launches this pre-pass and allocates this workspace on every
 *              call.
 *   unroll   : 1, 2 or 4; the reduction loop over MFMA k-steps is split by
 *              `unroll` and the inner part unrolled (tag "unr", sec. 2.4.2).
 *   precision: LPX_FP32 / LPX_BF16 / LPX_BF16X3.
 *   assume_tile_divides: 1 asserts E % tile_e == 0 (an assumption in the
 *              sense of sec. 2.1); a call whose E violates it fails with
 *              LPX_ERR_ASSUMPTION instead of computing.
 *   order    : how the outer loop of the split element loop (the tiles)
 *              is laid over the G persistent work-groups (loop order,
 *              sec. 2.3; split_iname, sec. 2.4.1): 0 = cyclic, work-group b
 *              takes tiles b, b + G, b + 2G, ... (neighbouring work-groups
 *              stream neighbouring tiles); 1 = blocked, work-group b takes
 *              the consecutive tiles b*c .. b*c + c - 1, c = ceil(ntiles /
 *              G) (each work-group streams one contiguous range).  The
 *              ragged batch lays out its own runs and ignores this field.
 *   gemm_tm, gemm_tn, gemm_tk: GEMM macro tile (rows of C, columns of C,
 *              reduction depth staged per step); 0 = library default.
 * Records are plain values (the paper's kernels are immutable, sec. 2.4):
 * the library never modifies one it is given.                          */
typedef struct lpx_record {
    uint32_t version;
    uint8_t precision;
    uint8_t tile_e;
    uint8_t prefetch;
    uint8_t unroll;
    uint8_t assume_tile_divides;
    uint8_t order;
    uint8_t reserved0[2];
    uint16_t gemm_tm;
    uint16_t gemm_tn;
    uint16_t gemm_tk;
    uint16_t reserved1;
} lpx_record;

/* The problem a record is chosen for. */
typedef struct lpx_problem {
    int32_t K;
    int32_t Np;
    int64_t E;
    int32_t layout;    /* LPX_ELEMENT_MAJOR / LPX_DOF_MAJOR */
    int32_t precision; /* the caller's accuracy class      */
} lpx_problem;

/* -------------------------------------------------------- contraction */
typedef struct lpx_contract_desc {
    int32_t K;        /* number of operators, >= 0                      */
    int32_t Np;       /* operator order (nodes per element), 0..128     */
    int64_t E;        /* number of elements, >= 0                       */
    int32_t layout;   /* LPX_ELEMENT_MAJOR / LPX_DOF_MAJOR              */
    int32_t reserved; /* must be 0                                      */
    const float* D;   /* device, K*Np*Np floats, 16-byte aligned        */
    const float* u;   /* device, E*Np floats, 16-byte aligned           */
    float* out;       /* device, K*E*Np floats, 16-byte aligned; must   */
                      /* not overlap D or u                             */
} lpx_contract_desc;

/* ------------------------------------------------- dG volume term */
/* Volume term of a nodal discontinuous Galerkin operator (Table 1's "dG
 * FEM volume" workload; the paper names the workload only).  Reading used
 * here: the K reference derivatives of each element are combined with that
 * element's geometric factors (derivatives of the reference coordinates
 * with respect to the physical ones),
 *
 *     out[d,e,i] = sum_{k<K} G(e,d,k) * sum_j D[k][i][j] * u[e][j],  d < K.
 *
 * Layouts as for the contraction (out like its output, K physical
 * derivatives in place of K reference ones), and G follows the layout:
 *   ELEMENT_MAJOR: G(e,d,k) = G[(e*K + d)*K + k]   (a K x K matrix per element)
 *   DOF_MAJOR    : G(e,d,k) = G[(d*K + k)*E + e]   (K*K runs of E factors)  */
#define LPX_DG_MAX_K 3
typedef struct lpx_dg_volume_desc {
    int32_t K;        /* reference = physical dimensions, 0..3            */
    int32_t Np;       /* nodes per element, 0..128                        */
    int64_t E;        /* number of elements, >= 0                         */
    int32_t layout;   /* LPX_ELEMENT_MAJOR / LPX_DOF_MAJOR                */
    int32_t reserved; /* must be 0                                        */
    const float* D;   /* device, K*Np*Np floats, 16-byte aligned          */
    const float* u;   /* device, E*Np floats, 16-byte aligned             */
    const float* G;   /* device, E*K*K floats, 16-byte aligned            */
    float* out;       /* device, K*E*Np floats, 16-byte aligned; must not */
                      /* overlap D, u or G                                */
} lpx_dg_volume_desc;

/* ------------------------------------------------ dG surface term */
/* Surface term of a nodal discontinuous Galerkin operator (Table 1's "dG
 * FEM surface"; named only).  Reading used here: each element's face
 * fluxes (nf faces of nfp nodes, M = nf*nfp values) are scaled by a factor
 * per face (the surface-to-volume Jacobian ratio of an affine element) and
 * lifted into the element's Np nodes by one rectangular operator L:
 *
 *     out[e,i] = sum_{m<M} L[i][m] * fl32(s(e, m / nfp) * f(e, m))
 *
 * (the product of factor and flux rounded to FP32, then the operands
 * treated per precision as for the contraction).  Storage:
 *   ELEMENT_MAJOR: f[e*M + m], s[e*nf + c], out[e*Np + i];
 *   DOF_MAJOR    : f[m*E + e], s[c*E + e], out[i*E + e].
 * L is L[i*M + m] in both.                                               */
typedef struct lpx_dg_surface_desc {
    int32_t Np;       /* nodes per element, 0..128                        */
    int32_t nf;       /* faces per element, >= 0                          */
    int32_t nfp;      /* nodes per face, >= 0; nf*nfp <= 4096             */
    int32_t layout;   /* LPX_ELEMENT_MAJOR / LPX_DOF_MAJOR                */
    int64_t E;        /* number of elements, >= 0                         */
    int32_t reserved; /* must be 0                                        */
    int32_t reserved2;/* must be 0                                        */
    const float* L;   /* device, Np*M floats, 16-byte aligned             */
    const float* f;   /* device, E*M floats, 16-byte aligned              */
    const float* s;   /* device, E*nf floats, 16-byte aligned             */
    float* out;       /* device, E*Np floats, 16-byte aligned; must not   */
                      /* overlap L, f or s                                */
} lpx_dg_surface_desc;

/* --------------------------------------------- 3D Coulomb potential */
/* phi[t] = sum over sources s with r_ts > 0 of q_s / r_ts, r_ts = |x_t - y_s|
 * (Table 1's "3D Coulomb pot." workload; the paper names it only).  Storage
 * (sec. 2.4.3, array of structures vs structure of arrays):
 *   ELEMENT_MAJOR (AoS): target t at targets[4t .. 4t+2] (4t+3 unused),
 *                        source s at sources[4s .. 4s+3] = (x, y, z, q);
 *   DOF_MAJOR     (SoA): targets[c*nt + t], c < 3; sources[f*ns + s], f < 4. */
typedef struct lpx_coulomb_desc {
    int64_t nt;             /* targets, 0 .. 2^40                          */
    int64_t ns;             /* sources, 0 .. 2^40                          */
    int32_t layout;         /* LPX_ELEMENT_MAJOR / LPX_DOF_MAJOR            */
    int32_t reserved;       /* must be 0                                    */
    const float* targets;   /* device; AoS 16-byte aligned, SoA 4-byte      */
    const float* sources;   /* device; as targets                           */
    float* phi;             /* device, nt floats; must not overlap inputs   */
} lpx_coulomb_desc;

/* -------------------------------------------------------------- GEMM */
/* C = A B, row-major FP32 (the degenerate case of the contraction). */
typedef struct lpx_gemm_desc {
    int64_t M, N, K;  /* C is M x N, A is M x K, B is K x N; each >= 0       */
    const float* A;   /* device; row m at A + m*lda; 16-byte aligned        */
    int64_t lda;      /* >= K (rows 16-byte aligned when a multiple of 4)   */
    const float* B;   /* device; row k at B + k*ldb; 16-byte aligned        */
    int64_t ldb;      /* >= N                                               */
    float* C;         /* device; row m at C + m*ldc; 16-byte aligned; must  */
    int64_t ldc;      /* not overlap A or B; ldc >= N                       */
} lpx_gemm_desc;

/* ------------------------------------------------------ support calls */
/* Library version string, e.g. "lpx 0.1.0 gfx950". */
const char* lpx_version(void);

/* Static text for a status code. */
const char* lpx_status_string(lpx_status s);

/* Text of the last failure on the calling thread ("" if none).  Valid until
 * the next lpx call on this thread. */
const char* lpx_last_error(void);

/* The untuned default record for a precision: tile_e = 16, prefetch = 0,
 * unroll = 1 (one 16x16 output block per MFMA chain, operands straight from
 * global memory), GEMM tiles 0 (library default).  `out` is host memory. */
lpx_status lpx_record_default(int32_t precision, lpx_record* out);

/* Checks a record's fields (version, ranges); LPX_OK if well formed. */
lpx_status lpx_record_validate(const lpx_record* rec);

/* Human-readable one-line description of a record, NUL-terminated, into
 * the host buffer `buf` of `len` bytes (truncated if short). */
lpx_status lpx_record_describe(const lpx_record* rec, char* buf, size_t len);

/* The candidate records of a problem in canonical order: precision fixed to
 * p->precision, then order in {0,1} (outermost), tile_e in {16,32,64},
 * prefetch in {0,1,2,3,4,6,10,11,14}, unroll in {1,2,4} (inner):
 * LPX_MAX_RECORDS = 162 records (some may be unsupported for a given
 * shape; the first 81 are the cyclic-order ones).  Writes min(cap, 162)
 * records to the host array `recs` and the total count to *n. */
#define LPX_MAX_RECORDS 162
lpx_status lpx_record_enumerate(const lpx_problem* p, lpx_record* recs,
                                int32_t cap, int32_t* n);

/* Dynamic LDS bytes one work-group of the record's kernel uses for the
 * problem (0 when prefetch = 0); LPX_ERR_UNSUPPORTED if it exceeds the
 * gfx950 limit, which is what lpx_contract would return. */
lpx_status lpx_contract_lds_bytes(const lpx_problem* p, const lpx_record* rec,
                                  int64_t* bytes);

/* ------------------------------------------------------- entry points */
/* Batched dense contraction  out[k,e,i] = sum_j D[k][i][j] u[e][j]
 * (the reduction of sec. 2.1 applied per element; Table 1 "dG FEM
 * volume"), enqueued on `stream`.  `rec` selects the code variant; NULL
 * means the untuned default of precision FP32.  Every output element is
 * written exactly once; nothing outside `out` is written.  Summation order
 * is the variant's own (the programming model is unordered, sec. 2.3), so
 * results of different records agree to rounding, and bit for bit when all
 * partial sums are exact.  Records that read D from memory (prefetch bits 0
 * and 2 clear, the untuned default among them) launch a pre-pass kernel
 * that writes D's MFMA-order arrangement into a workspace allocated on
 * `stream` from the library's own memory pool, and free it after the
 * kernel; the others allocate nothing and launch one kernel. */
lpx_status lpx_contract(const lpx_contract_desc* c, const lpx_record* rec,
                        void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * contraction as lpx_contract, with the same kernels and bit-identical
 * results, but no allocation of any kind (no hipMalloc, hipFree or
 * stream-ordered allocation).  Records that read D from memory (prefetch
 * bits 0 and 2 clear, the untuned default among them) write D's MFMA-order
 * arrangement into a static scratch array of LPX_NOALLOC_SCRATCH_BYTES in
 * device memory instead of a per-call workspace; each GPU the library runs
 * on holds its own copy of that array until the process ends.  The
 * arrangement takes nrb*nsteps*64 fragments of 4 (FP32), 16 (BF16) or 32
 * (BF16X3) bytes, nrb = ceil(K*Np/16), nsteps = ceil(Np/4) for FP32 and
 * ceil(Np/32) otherwise (K = 3, Np = 128: 192 KiB in every precision); a
 * problem whose arrangement is larger fails with LPX_ERR_UNSUPPORTED before
 * any HIP call.  Other records use no scratch.  Every call on a GPU shares
 * that GPU's array and nothing in it needs clearing (each call rewrites
 * what it reads): calls that overlap on one GPU -- on different streams,
 * or from threads without ordering between them -- race on it and may
 * return wrong results.  The first call on a device looks up the array's
 * device address (hipGetSymbolAddress).  Errors as for lpx_contract. */
#define LPX_NOALLOC_SCRATCH_BYTES 1048576
lpx_status lpx_contract_noalloc(const lpx_contract_desc* c, const lpx_record* rec,
                                void* stream);

/* Runs every check lpx_contract makes before enqueueing (arguments,
 * record, assumption, aliasing, LDS budget) and returns the status
 * lpx_contract would return for them, without any HIP call and without
 * reading through the pointers.  Device-dependent failures (LPX_ERR_HIP)
 * can still occur in lpx_contract after this returns LPX_OK. */
lpx_status lpx_contract_validate(const lpx_contract_desc* c, const lpx_record* rec);

/* The dG volume term (see lpx_dg_volume_desc), enqueued on `stream`, with
 * the metric applied in the write-back: the contraction's compute waves
 * stage the K reference derivatives of an element tile in LDS exactly as
 * lpx_contract's staged-output records do (same kernels, same summation
 * order), together with the tile's geometric factors, and the store waves
 * form out[d] = sum_k G(e,d,k) * (D_k u)[i] (FP32, k in increasing order)
 * while they copy the tile to `out`.  So the record must stage the output
 * tile: prefetch 10, 11 or 14 (bit 3), any tile_e, unroll and precision;
 * other records fail with LPX_ERR_UNSUPPORTED, as do K > 3 and shapes
 * whose LDS rings do not fit.  rec = NULL picks the first of (tile_e,
 * prefetch) = (64, 14), (64, 10), (32, 10), (16, 10) that fits, in FP32.
 * Records that read D from memory (prefetch 10) launch the D-arrangement
 * pre-pass with its workspace, as lpx_contract does.  Errors as for
 * lpx_contract; G must not overlap out. */
lpx_status lpx_dg_volume(const lpx_dg_volume_desc* c, const lpx_record* rec, void* stream);

/* Every pre-launch check of lpx_dg_volume, without any HIP call; with
 * rec = NULL, *chosen (host, may be NULL) receives the record NULL stands
 * for. */
lpx_status lpx_dg_volume_validate(const lpx_dg_volume_desc* c, const lpx_record* rec,
                                  lpx_record* chosen);

/* The dG surface (lift) term, enqueued on `stream`: the contraction with a
 * rectangular operator and the per-face scaling fused into the operand
 * reads.  Record: precision FP32, BF16 or BF16X3; prefetch must be 1 (the
 * operator is staged in LDS once per work-group, in MFMA operand order, up
 * to 160 KiB: Np = 128 allows M up to 320), else LPX_ERR_UNSUPPORTED;
 * tile_e / 16 element blocks go to each wave at a time, so each operator
 * fragment read from LDS feeds that many MFMAs; unroll does not apply.
 * rec = NULL: FP32, tile_e 16, prefetch 1.  Every record of a precision
 * sums each output in column order with the same operations (bit-identical
 * results).  Zero sizes are no-ops. */
lpx_status lpx_dg_surface(const lpx_dg_surface_desc* c, const lpx_record* rec, void* stream);

/* Every pre-launch check of lpx_dg_surface, without any HIP call. */
lpx_status lpx_dg_surface_validate(const lpx_dg_surface_desc* c, const lpx_record* rec);

/* The Coulomb potential, enqueued on `stream`.  The record is the
 * variant: tile_e sets the source tile (16 * tile_e = 256, 512 or 1024
 * sources, split_iname of the source loop, sec. 2.4.1), prefetch 2 stages
 * each tile in LDS (add_prefetch, sec. 2.4.4) and 0 reads sources from
 * global memory at one address per wave, unroll is the number of targets
 * per thread (the `ilp` tag, sec. 2.4.2); precision must be FP32 and other
 * prefetch values fail with LPX_ERR_UNSUPPORTED.  rec = NULL: tile_e 16,
 * prefetch 0, unroll 1.  Each target sums its pairs in increasing source
 * order in FP32 (reciprocal square root v_rsq_f32, fused multiply-adds), so
 * every record gives bit-identical results.  A pair at zero distance
 * contributes nothing.  nt = 0 is a no-op; ns = 0 writes zeros. */
lpx_status lpx_coulomb(const lpx_coulomb_desc* c, const lpx_record* rec, void* stream);

/* Every pre-launch check of lpx_coulomb, without any HIP call. */
lpx_status lpx_coulomb_validate(const lpx_coulomb_desc* c, const lpx_record* rec);

/* Dense GEMM  C[m][n] = sum_k A[m][k] B[k][n]  (the paper's sec. 2.1
 * reduction example sum(k, a[i,k]*b[k,j]); Table 1 "sgemm"), enqueued on
 * `stream`.  The record supplies the precision (as for lpx_contract; the
 * products follow the same FP32 / BF16 / BF16X3 rules, FP32 accumulation)
 * and the tiling: gemm_tm x gemm_tn tile of C per work-group, gemm_tk-deep
 * k slabs staged in LDS (0 = 128 x 128 x 32 for FP32, 128 x 128 x 64 for
 * BF16, and for BF16X3 256 x 256 x 32 when ceil(M/256) ceil(N/256) >= 256,
 * else 128 x 128 x 64).  Built tilings: 64x64x32, 64x64x64, 128x128x32,
 * 128x128x64, 128x64x32, 64x128x32; for FP32/BF16 also 256x128x32,
 * 128x256x32, 256x256x32; for BF16 also 256x256x64, 256x128x64; for BF16X3
 * also 256x256x32, 256x128x32; others return LPX_ERR_UNSUPPORTED.  BF16 /
 * BF16X3 at 128x128x64 and at the 256-row tilings (with K > 0) first split
 * both operands once into K-contiguous bf16 planes (B transposed) in
 * stream-ordered workspace (allocated on `stream` from the library's own
 * memory pool, freed the same way), then stream the planes into LDS with
 * direct global-to-LDS loads; the other tilings convert the FP32 operands
 * slab by slab.  C is overwritten (no alpha/beta).  rec = NULL means FP32
 * with the default tiling.  Errors as for lpx_contract. */
lpx_status lpx_gemm(const lpx_gemm_desc* g, const lpx_record* rec, void* stream);

/* Every pre-launch check of lpx_gemm, without any HIP call. */
lpx_status lpx_gemm_validate(const lpx_gemm_desc* g, const lpx_record* rec);

/* Split-precision conversion: hi[t] = bf16(x[t]), lo[t] = bf16(x[t] -
 * float(hi[t])), round-to-nearest-even, as raw bfloat16 bit patterns.
 * x, hi, lo are device pointers of n elements (x 4-byte, hi/lo 2-byte
 * aligned); hi and lo must not overlap x or each other.  This is the
 * operand transformation behind LPX_BF16 (hi only) and LPX_BF16X3. */
lpx_status lpx_split_bf16(const float* x, uint16_t* hi, uint16_t* lo,
                          int64_t n, void* stream);

/* ------------------------------------------------------- ragged batch */
/* Many contractions of uneven sizes in one HIP graph (one persistent
 * launch per kernel the records select), captured once and replayed.
 * Opaque, library-owned handle. */
typedef struct lpx_batch lpx_batch;

/* items[0..n-1]: contraction descriptors (validated as by lpx_contract; no
 * zero sizes).  recs: one record per item, or NULL to take each item's FP32
 * winner from the tuning cache, else the FP32 default.  Every record is
 * honoured: each instance is checked as lpx_contract would check it with
 * its record (a record whose storage does not fit the instance fails the
 * call, naming the instance) and runs that record's kernel, so instances
 * may differ in precision, layout and every record field.
 *   *h == NULL: builds the batch and launches it on `stream`, returning the
 *     handle in *h.  Instances are grouped by the kernel their record
 *     selects; each group is one persistent launch of that kernel's batch
 *     form, which runs the contraction's own tile code on runs of
 *     consecutive element tiles of one instance at a time (D staged or
 *     loaded again at the start of a run).  Each instance's tiles are cut
 *     into runs of similar length, and the runs are dealt largest first to
 *     the least-loaded work-group.  Records that read D from memory get its
 *     MFMA-order arrangement from the graph's first nodes (into device
 *     memory the batch owns).  The nodes are captured once into a HIP graph,
 *     the group launches on four parallel branches.
 *   *h != NULL, items != NULL: items must have the batch's n and per-item
 *     K, Np, E and layout (pointers may change); copies the updated
 *     descriptor table and replays the graph on `stream`.
 *   *h != NULL, items == NULL: replays the graph on `stream` with the
 *     table of the last submit (no host-side work, no copy; recs and n are
 *     not read).
 * Outputs are bit-identical to lpx_contract with the same records (and to
 * any record of the same precision: every record of a precision sums each
 * output in the same order).  The caller keeps all buffers alive until
 * `stream` passes the work. */
lpx_status lpx_batch_submit(const lpx_contract_desc* items, const lpx_record* recs,
                            int32_t n, lpx_batch** h, void* stream);

/* Batch autotuner: the instances are grouped by (K, Np, layout); for each
 * group every cyclic-order candidate record of `precision`
 * (lpx_record_enumerate order; the batch ignores the tile order, so the
 * blocked-order copies are not timed) that fits all of the group's
 * instances is timed on the group alone, as a
 * batch built with that record for each of them -- `warmup` untimed
 * replays, then `reps` replays bracketed by HIP events on `stream`, median
 * kept -- and recs_out[i] (host array of n) receives the fastest record of
 * instance i's group (ties: lowest index).  The records a batch needs
 * differ from the ones separate calls need: in a batch the other instances
 * fill the GPU, so a small instance no longer wants small tiles.  Blocks
 * the calling thread; overwrites every out buffer; allocates and frees
 * device memory per candidate. */
lpx_status lpx_batch_tune(const lpx_contract_desc* items, int32_t n, int32_t precision,
                          int32_t warmup, int32_t reps, void* stream, lpx_record* recs_out);

/* Element tiles in the batch (each instance cut by its record's tile_e),
 * kernels launched (one per group), work-groups over all launches and the
 * largest dynamic LDS of a launch (any output pointer may be NULL). */
lpx_status lpx_batch_info(const lpx_batch* b, int64_t* total_tiles, int32_t* kernels,
                          int32_t* grid, int64_t* lds_bytes);

/* Frees the batch; the caller must first make sure no submitted replay is
 * still running.  NULL is a no-op. */
lpx_status lpx_batch_destroy(lpx_batch* b);

/* ------------------------------------------------ variant selection */
/* Exhaustive autotuner: times every candidate record of the problem
 * (lpx_record_enumerate order) on the caller's buffers -- `warmup` untimed
 * launches, then `reps` launches each bracketed by HIP events on `stream`,
 * median kept -- and returns the fastest in *best (ties: lowest index).
 * If flush (device, flush_bytes, a multiple of 16) is not NULL it is
 * overwritten before every timed launch, outside the events, so that the
 * caches hold none of the problem's data, only dirty lines of the flush
 * buffer (as after other work; needed for problems that fit the
 * last-level cache).
 * Blocks the calling thread until the timing launches finish.  Overwrites
 * c->out.  Candidates that lpx_contract_validate rejects (e.g. LDS budget)
 * are skipped and reported as +infinity.  Writes min(cap, count) median
 * times in microseconds to the host array times_us and the count to *n
 * (n may be NULL).  The winner is also stored in the library's tuning
 * cache, keyed by (device, K, Np, E, layout, precision), where
 * LPX_PICK_EXHAUSTIVE finds it. */
lpx_status lpx_autotune(const lpx_contract_desc* c, int32_t precision, int32_t warmup,
                        int32_t reps, void* flush, int64_t flush_bytes, void* stream,
                        lpx_record* best, float* times_us, int32_t cap, int32_t* n);

/* Seeds the tuning cache for the current device (e.g. from a stored timing
 * database); the record's precision must equal p->precision. */
lpx_status lpx_tune_cache_insert(const lpx_problem* p, const lpx_record* rec);

/* Empties the tuning cache. */
lpx_status lpx_tune_cache_clear(void);

/* --------------------------------------------------- learned picker */
/* Cost model: a perceptron 13 -> 64 -> 64 -> 1 with ReLU hidden units that
 * predicts the log run time of one (problem, record) pair.  Parameters are
 * one flat FP32 vector: W1[64][13], b1[64], W2[64][64], b2[64], w3[64], b3.
 * Every kernel below sums in a fixed order (deterministic results). */
#define LPX_MLP_FEATURES 13
#define LPX_MLP_HIDDEN 64
#define LPX_MLP_PARAMS 5121

/* The 13 features of (problem, record), into the host array out[13]:
 * log2 Np, log2 E, K, layout, log2 tile_e, D storage, staging (0 none,
 * 1 u tile, 2 u and output tiles), log2 unroll, precision code, MFMA row
 * padding of the stacked operator rows (16*ceil(K*Np/16) - K*Np) /
 * (16*ceil(K*Np/16)), alignment class 2*(Np % 4 == 0) + (E % 4 == 0)
 * (vector or scalar row and element accesses), dynamic LDS bytes per
 * work-group / 160 KiB, tile order (0 cyclic, 1 blocked).  The
 * D-prefetch feature is the storage of D:
 * 0 global, 1 LDS, 2 registers.  Needs 0 < K, 0 < Np <= 128, 0 < E. */
lpx_status lpx_features(const lpx_problem* p, const lpx_record* r, float* out);

/* Forward pass of n rows.  params: device, LPX_MLP_PARAMS floats; X: device
 * n x 13; act: device n x 128 (per row z1[64] then z2[64], kept for the
 * backward pass) or NULL; y: device n predictions. */
lpx_status lpx_mlp_forward(const float* params, const float* X, int32_t n, float* act,
                           float* y, void* stream);

/* Mean squared error L = mean((y - t)^2) into loss[0] (device, may be NULL)
 * and its gradient dy = 2 (y - t) / n (device n floats, may be NULL);
 * n > 0. */
lpx_status lpx_mlp_loss(const float* y, const float* t, int32_t n, float* dy, float* loss,
                        void* stream);

/* Backward pass: grads (device, LPX_MLP_PARAMS) = gradient of
 * sum_b dy[b] * y[b] with respect to the parameters (ReLU'(0) = 0), from the
 * forward pass's X and act; work: device n x 128 scratch. */
lpx_status lpx_mlp_backward(const float* params, const float* X, const float* act,
                            const float* dy, int32_t n, float* work, float* grads, void* stream);

/* One Adam update of n parameters in place (device m, v moments), with
 * bias correction for `step` (>= 1): p -= lr * mhat / (sqrt(vhat) + eps). */
lpx_status lpx_adam_step(float* params, const float* grads, float* m, float* v, int32_t n,
                         int32_t step, float lr, float beta1, float beta2, float eps,
                         void* stream);

/* Pick kernel: standardises ncand (1..256) candidate feature rows (device
 * ncand x 12) with mean/std (device, 12 each; std 0 counts as 1), predicts
 * each (pred: device ncand floats or NULL) and writes the argmin index to
 * best (device int; ties: lowest index). */
lpx_status lpx_mlp_pick(const float* params, const float* feats, int32_t ncand,
                        const float* mean, const float* stdv, float* pred, int32_t* best,
                        void* stream);

/* A trained picker: weights plus feature standardisation, loaded from a
 * model file (magic "LPXPICK1", version, dimensions, mean[13], std[13],
 * params[5121], FNV-1a checksum; little-endian).  Opaque. */
typedef struct lpx_picker lpx_picker;

/* Writes a model file from host arrays. */
lpx_status lpx_picker_save(const char* path, const float* params, const float* mean,
                           const float* stdv);
/* Loads a model file; LPX_ERR_MODEL if it is missing, truncated, of another
 * version or dimensions, fails its checksum, or holds non-finite values. */
lpx_status lpx_picker_load(const char* path, lpx_picker** out);
/* Copies a loaded picker's weights/standardisation to host arrays (any may
 * be NULL). */
lpx_status lpx_picker_params(const lpx_picker* m, float* params, float* mean, float* stdv);
lpx_status lpx_picker_free(lpx_picker* m);

#define LPX_PICK_UNTUNED 0    /* the default record                     */
#define LPX_PICK_EXHAUSTIVE 1 /* the tuning cache (LPX_ERR_NOT_TUNED)   */
#define LPX_PICK_LEARNED 2    /* the cost model's argmin                */

/* Chooses a record of p->precision for the problem.  LEARNED enumerates the
 * candidates that fit (lpx_record_enumerate minus LDS misfits), computes
 * their features on the host, runs lpx_mlp_pick on `stream` and waits for
 * the index (a blocking round trip; the answer is cached per problem in the
 * picker).  model is needed only for LEARNED (LPX_ERR_MODEL if NULL). */
lpx_status lpx_pick_variant(const lpx_problem* p, int32_t mode, lpx_picker* model,
                            void* stream, lpx_record* out);

/* ------------------------------------------------------ measurement */
/* Streaming probe, the analogue of Table 1's "saxpy" row: y[r*n + t] =
 * x[t] for r < fanout (fanout 1 = plain copy; fanout 3 = the contraction's
 * one-read-three-writes byte mix).  x: device, n floats; y: device,
 * fanout*n floats; n a multiple of 4, pointers 16-byte aligned, y must not
 * overlap x.  Used to measure the achievable HBM rate and to calibrate
 * hardware byte counters against a kernel of known traffic. */
lpx_status lpx_stream_probe(const float* x, float* y, int64_t n, int32_t fanout, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LPX_H */
