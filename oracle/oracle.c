/*
 * oracle.c -- plain FP64 CPU reference for the batched dense contraction
 * and its degenerate case, dense GEMM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * GPU path.
 *
 * What it computes (Klöckner, "Loo.py: transformation-based code generation
 * for GPUs and CPUs", ARRAY'14):
 *
 *   - the reduction  sum(j, D[k,i,j] * u[e,j])  written in the paper's
 *     reduction syntax (sec. 2.1, which admits reductions in instructions), i.e. the
 *     element-local operator application behind Table 1's "dG FEM volume"
 *     row:   out[k,e,i] = sum_j D[k][i][j] * u[e][j];
 *   - its degenerate case C[m,n] = sum_k A[m,k]*B[k,n], the paper's own
 *     reduction example sum(k, a[i,k]*b[k,j]) and Table 1's "sgemm" row.
 *
 * Every transformation the method offers (tiling, prefetch, unrolling,
 * data-layout change) preserves this result up to summation order, because
 * the programming model is unordered (sec. 2.3): a program must give a
 * valid result for any traversal order.  So the oracle is the definition
 * itself: a plain loop, FP64 accumulation, j in increasing order.
 *
 * Precision modes.  The paper generates code for the runtime type of the
 * arguments (sec. 2.1/2.2: one variant per type combination) and leaves
 * semantics-changing choices to the user.  Reduced-precision products are
 * such a user choice; the oracle emulates them by rounding the operands
 * the same way before the exact FP64 product:
 *   PREC_FP32   : D * u
 *   PREC_BF16   : bf16(D) * bf16(u)
 *   PREC_BF16X3 : hi_D*hi_u + hi_D*lo_u + lo_D*hi_u,
 *                 hi = bf16(x), lo = bf16(x - hi)   (lo*lo dropped)
 * bf16() is round-to-nearest-even on the FP32 bit pattern.
 *
 * Layouts (sec. 2.4.3, array-axis implementation tags):
 *   LAYOUT_EM (element-major): u[e*Np + j],  out[(k*E + e)*Np + i]
 *   LAYOUT_DM (DOF-major)    : u[j*E + e],   out[(k*Np + i)*E + e]
 * The oracle's output is always the chunk ref[k][e - e0][i] (FP64) for
 * e in [e0, e0 + ne), whatever the input layout, so a caller can compare
 * a huge GPU output chunk by chunk or at sampled elements.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PREC_FP32 0
#define PREC_BF16 1
#define PREC_BF16X3 2
#define LAYOUT_EM 0
#define LAYOUT_DM 1

int oracle_version(void) { return 1; }

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Round an FP32 value to the nearest bfloat16 (ties to even), returned as
 * the FP32 value it represents.  bfloat16 keeps the sign, the 8 exponent
 * bits and the top 7 mantissa bits of an IEEE binary32, so rounding is done
 * on the low 16 bits of the pattern.  NaN stays NaN (made quiet). */
float oracle_bf16_rne(float x) {
    uint32_t b;
    memcpy(&b, &x, sizeof b);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu) != 0) {
        b = (b | 0x00400000u) & 0xffff0000u;  /* quiet NaN, top payload */
    } else {
        uint32_t low = b & 0xffffu;
        uint32_t keep = b & 0xffff0000u;
        uint32_t lsb = (keep >> 16) & 1u;
        if (low > 0x8000u || (low == 0x8000u && lsb)) keep += 0x10000u;
        b = keep;                     /* a carry into the exponent is right */
    }
    float r;
    memcpy(&r, &b, sizeof r);
    return r;
}

/* hi = bf16(x); lo = bf16(x - hi).  x - hi is exact in FP32 (hi shares
 * x's exponent range and the difference fits in the mantissa). */
void oracle_split_bf16(const float* x, float* hi, float* lo, long n) {
    for (long t = 0; t < n; ++t) {
        float h = oracle_bf16_rne(x[t]);
        hi[t] = h;
        lo[t] = oracle_bf16_rne(x[t] - h);
    }
}

/* The product a*b under a precision mode, evaluated exactly in FP64
 * (a product of two FP32 values has at most 48 significant bits). */
static double prod(float a, float b, int precision) {
    if (precision == PREC_FP32) return (double)a * (double)b;
    if (precision == PREC_BF16)
        return (double)oracle_bf16_rne(a) * (double)oracle_bf16_rne(b);
    float ah = oracle_bf16_rne(a), bh = oracle_bf16_rne(b);
    float al = oracle_bf16_rne(a - ah), bl = oracle_bf16_rne(b - bh);
    return (double)ah * (double)bh + (double)ah * (double)bl +
           (double)al * (double)bh;
}

/* ref[k][e - e0][i] = sum_{j=0}^{Np-1} D[k][i][j] * u(e, j), FP64. */
void oracle_contract(int K, int Np, long E, int layout, int precision,
                     const float* D, const float* u, long e0, long ne,
                     double* ref) {
    if (K <= 0 || Np <= 0 || ne <= 0) return;
#pragma omp parallel for schedule(static)
    for (long de = 0; de < ne; ++de) {
        long e = e0 + de;
        for (int k = 0; k < K; ++k) {
            const float* Dk = D + (long)k * Np * Np;
            for (int i = 0; i < Np; ++i) {
                double acc = 0.0;
                for (int j = 0; j < Np; ++j) {
                    float uej = (layout == LAYOUT_EM) ? u[e * Np + j]
                                                      : u[(long)j * E + e];
                    acc += prod(Dk[(long)i * Np + j], uej, precision);
                }
                ref[((long)k * ne + de) * Np + i] = acc;
            }
        }
    }
}

/* Volume term of a nodal discontinuous Galerkin operator (the "dG FEM
 * volume" workload of Table 1; the paper names it and prints nothing else
 * about it).  Reading: the K reference derivatives D_k u of an element are
 * combined with that element's geometric factors (the derivatives of the
 * reference coordinates with respect to the physical ones),
 *
 *   ref[d][e - e0][i] = sum_{k<K} G(e, d, k) * sum_{j<Np} D[k][i][j] * u(e, j),
 *
 * d < K, with G(e, d, k) = G[(e*K + d)*K + k] for element-major storage
 * and G[(d*K + k)*E + e] for DOF-major storage (one contiguous run of E
 * factors per (d, k), like u's rows).  The inner sums are oracle_contract's,
 * under the same precision mode; the factors are applied in FP64 to the
 * FP64 sums.  K <= 8. */
void oracle_dg_volume(int K, int Np, long E, int layout, int precision,
                      const float* D, const float* u, const float* G, long e0,
                      long ne, double* ref) {
    if (K <= 0 || K > 8 || Np <= 0 || ne <= 0) return;
#pragma omp parallel for schedule(static)
    for (long de = 0; de < ne; ++de) {
        long e = e0 + de;
        double t[8 * 128];  /* reference derivatives of element e, [k][i] */
        for (int k = 0; k < K; ++k) {
            const float* Dk = D + (long)k * Np * Np;
            for (int i = 0; i < Np; ++i) {
                double acc = 0.0;
                for (int j = 0; j < Np; ++j) {
                    float uej = (layout == LAYOUT_EM) ? u[e * Np + j]
                                                      : u[(long)j * E + e];
                    acc += prod(Dk[(long)i * Np + j], uej, precision);
                }
                t[k * Np + i] = acc;
            }
        }
        for (int d = 0; d < K; ++d) {
            for (int i = 0; i < Np; ++i) {
                double acc = 0.0;
                for (int k = 0; k < K; ++k) {
                    float g = (layout == LAYOUT_EM) ? G[(e * K + d) * K + k]
                                                    : G[((long)d * K + k) * E + e];
                    acc += (double)g * t[k * Np + i];
                }
                ref[((long)d * ne + de) * Np + i] = acc;
            }
        }
    }
}

/* Surface term of a nodal discontinuous Galerkin operator (the "dG FEM
 * surface" workload of Table 1; named only).  Reading: each element's face
 * fluxes (nf faces of nfp nodes, M = nf*nfp values) are scaled by a per-
 * face factor (the surface-to-volume Jacobian ratio of an affine element)
 * and lifted into the element's Np nodes by one rectangular operator
 * L [Np][M]:
 *
 *   ref[e - e0][i] = sum_{m < M} L[i][m] * (s(e, m / nfp) * f(e, m)),
 *
 * m in increasing order, FP64, the scaled value rounded to FP32 first (the
 * scaling is an FP32 product on the GPU); under a reduced-precision mode the
 * scaled FP32 value and L are the operands rounded as in prod().
 * Element-major: f(e, m) = f[e*M + m], s(e, c) = s[e*nf + c],
 * out[e*Np + i]; DOF-major: f[m*E + e], s[c*E + e], out[i*E + e]. */
void oracle_dg_surface(int Np, int nf, int nfp, long E, int layout, int precision,
                       const float* L, const float* f, const float* sc, long e0, long ne,
                       double* ref) {
    const long M = (long)nf * nfp;
    if (Np <= 0 || M <= 0 || ne <= 0) return;
#pragma omp parallel for schedule(static)
    for (long de = 0; de < ne; ++de) {
        long e = e0 + de;
        for (int i = 0; i < Np; ++i) {
            double acc = 0.0;
            for (long m = 0; m < M; ++m) {
                long c = m / nfp;
                float fv = (layout == LAYOUT_EM) ? f[e * M + m] : f[m * E + e];
                float sv = (layout == LAYOUT_EM) ? sc[e * nf + c] : sc[c * E + e];
                float g = sv * fv; /* FP32 product, as the GPU forms it */
                acc += prod(L[(long)i * M + m], g, precision);
            }
            ref[de * Np + i] = acc;
        }
    }
}

/* 3D Coulomb potential (Table 1's "3D Coulomb pot." workload, counted in
 * pairs per second; the paper names it only).  Reading: the potential at
 * each target point due to point charges at the source points,
 *
 *   ref[t - t0] = sum_{s < ns, r_ts > 0} q_s / r_ts,
 *   r_ts = |x_t - y_s| (Euclidean, 3D),
 *
 * sources in increasing index order, FP64; a source at the target's own
 * position (r = 0) contributes nothing.  Storage (the paper's array-of-
 * structures / structure-of-arrays layout switch): LAYOUT_EM = AoS, target
 * t at tg[4t .. 4t+2] (4t+3 unused), source s at sr[4s .. 4s+3] = (x, y, z,
 * q); LAYOUT_DM = SoA, target coordinate c at tg[c*nt + t], source field f
 * at sr[f*ns + s]. */
void oracle_coulomb(long nt, long ns, int layout, const float* tg, const float* sr, long t0,
                    long n, double* ref) {
    if (n <= 0) return;
#pragma omp parallel for schedule(static)
    for (long dt = 0; dt < n; ++dt) {
        long t = t0 + dt;
        double xt[3];
        for (int c = 0; c < 3; ++c)
            xt[c] = (layout == LAYOUT_EM) ? (double)tg[4 * t + c] : (double)tg[c * nt + t];
        double acc = 0.0;
        for (long s = 0; s < ns; ++s) {
            double r2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                double ys = (layout == LAYOUT_EM) ? (double)sr[4 * s + c] : (double)sr[c * ns + s];
                double d = xt[c] - ys;
                r2 += d * d;
            }
            double q = (layout == LAYOUT_EM) ? (double)sr[4 * s + 3] : (double)sr[3 * ns + s];
            if (r2 > 0.0) acc += q / sqrt(r2);
        }
        ref[dt] = acc;
    }
}

/* C[m - m0][n] = sum_{k=0}^{Kd-1} A[m][k] * B[k][n], A (M x Kd) and
 * B (Kd x N) row-major, FP64, for m in [m0, m0 + nm). */
void oracle_gemm(long M, long N, long Kd, int precision, const float* A,
                 const float* B, long m0, long nm, double* C) {
    (void)M;
    if (nm <= 0 || N <= 0) return;
#pragma omp parallel for schedule(static)
    for (long dm = 0; dm < nm; ++dm) {
        long m = m0 + dm;
        double* Crow = C + dm * N;
        for (long n = 0; n < N; ++n) Crow[n] = 0.0;
        for (long k = 0; k < Kd; ++k) {
            float a = A[m * Kd + k];
            const float* Brow = B + k * N;
            for (long n = 0; n < N; ++n) Crow[n] += prod(a, Brow[n], precision);
        }
    }
}
