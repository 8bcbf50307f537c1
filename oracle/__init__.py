"""FP64 CPU oracle for the batched dense contraction and GEMM.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no
code with the GPU path; the C part (``oracle.c``) is compiled with gcc.

Functions follow the plain definitions:
  * ``contract``  out[k,e,i] = sum_j D[k][i][j] u[e][j]   (paper sec. 2.1
    reduction syntax; Table 1 "dG FEM volume"), FP64 accumulation;
  * ``gemm``      C = A B                                   (sec. 2.1 example
    reduction sum(k, a[i,k]*b[k,j]); Table 1 "sgemm");
  * ``dg_volume`` out[d,e,i] = sum_k G(e,d,k) sum_j D[k][i][j] u[e][j]
    (Table 1 "dG FEM volume": reference derivatives combined with
    per-element geometric factors);
  * ``dg_surface`` out[e,i] = sum_m L[i][m] s(e,m/nfp) f(e,m) (Table 1 "dG
    FEM surface": face fluxes lifted by a rectangular operator);
  * ``coulomb``   phi[t] = sum_s q_s / |x_t - y_s|          (Table 1 "3D
    Coulomb pot."), FP64;
  * ``bf16_rne`` / ``split_bf16``  reduced-precision operand emulation;
  * ``mlp``       the cost model's forward, backward and Adam step (numpy).
"""
import ctypes
import os

import numpy as np

from .build import LIB, SRC, build

PREC = {"fp32": 0, "bf16": 1, "bf16x3": 2}
LAYOUT = {"em": 0, "dm": 1}

class Oracle:
    """ctypes handle on one build of ``oracle.c`` (the default build, or a
    mutated copy built by a test that checks the pins catch mistakes)."""

    def __init__(self, path):
        L = ctypes.CDLL(path)
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        L.oracle_bf16_rne.restype = ctypes.c_float
        L.oracle_bf16_rne.argtypes = [ctypes.c_float]
        L.oracle_split_bf16.argtypes = [f32p, f32p, f32p, ctypes.c_long]
        L.oracle_contract.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long,
                                      ctypes.c_int, ctypes.c_int, f32p, f32p,
                                      ctypes.c_long, ctypes.c_long, f64p]
        L.oracle_gemm.argtypes = [ctypes.c_long, ctypes.c_long, ctypes.c_long,
                                  ctypes.c_int, f32p, f32p, ctypes.c_long,
                                  ctypes.c_long, f64p]
        L.oracle_dg_volume.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long,
                                       ctypes.c_int, ctypes.c_int, f32p, f32p, f32p,
                                       ctypes.c_long, ctypes.c_long, f64p]
        L.oracle_dg_surface.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_long,
                                        ctypes.c_int, ctypes.c_int, f32p, f32p, f32p,
                                        ctypes.c_long, ctypes.c_long, f64p]
        L.oracle_coulomb.argtypes = [ctypes.c_long, ctypes.c_long, ctypes.c_int, f32p, f32p,
                                     ctypes.c_long, ctypes.c_long, f64p]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        self.L = L

    def threads(self) -> int:
        return self.L.oracle_threads()

    def set_threads(self, n: int) -> None:
        self.L.oracle_set_threads(int(n))

    def split_bf16(self, x):
        """(hi, lo): hi = bf16(x), lo = bf16(x - hi), as FP32 arrays."""
        x, px = _f32(x)
        hi = np.empty_like(x)
        lo = np.empty_like(x)
        fp = ctypes.POINTER(ctypes.c_float)
        self.L.oracle_split_bf16(px, hi.ctypes.data_as(fp), lo.ctypes.data_as(fp),
                                 x.size)
        return hi, lo

    def bf16_rne(self, x):
        """Round FP32 values to bfloat16 (nearest, ties to even)."""
        return self.split_bf16(x)[0]

    def contract(self, D, u, layout="em", precision="fp32", e0=0, ne=None):
        """FP64 reference chunk ref[k, e - e0, i] for e in [e0, e0 + ne).

        D: (K, Np, Np) float32.  u: (E, Np) for layout "em", (Np, E) for "dm".
        """
        D, pD = _f32(D)
        K, Np, Np2 = D.shape
        assert Np == Np2
        u, pu = _f32(u)
        E = u.shape[0] if layout == "em" else u.shape[1]
        assert (u.shape[1] if layout == "em" else u.shape[0]) == Np
        if ne is None:
            ne = E - e0
        assert 0 <= e0 and e0 + ne <= E
        ref = np.zeros((K, ne, Np), dtype=np.float64)
        self.L.oracle_contract(K, Np, E, LAYOUT[layout], PREC[precision], pD, pu,
                               e0, ne,
                               ref.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return ref

    def dg_volume(self, D, u, G, layout="em", precision="fp32", e0=0, ne=None):
        """FP64 dG volume chunk ref[d, e - e0, i] = sum_k G(e,d,k) (D_k u_e)_i.

        G: (E, K, K) float32 for layout "em", (K, K, E) for "dm"."""
        D, pD = _f32(D)
        K, Np, Np2 = D.shape
        assert Np == Np2 and 0 < K <= 8 and Np <= 128
        u, pu = _f32(u)
        G, pG = _f32(G)
        E = u.shape[0] if layout == "em" else u.shape[1]
        assert G.shape == ((E, K, K) if layout == "em" else (K, K, E))
        if ne is None:
            ne = E - e0
        assert 0 <= e0 and e0 + ne <= E
        ref = np.zeros((K, ne, Np), dtype=np.float64)
        self.L.oracle_dg_volume(K, Np, E, LAYOUT[layout], PREC[precision], pD, pu, pG, e0, ne,
                                ref.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return ref

    def dg_surface(self, L, f, sc, nf, layout="em", precision="fp32", e0=0, ne=None):
        """FP64 lift chunk ref[e - e0, i] = sum_m L[i][m] fl32(s(e, m // nfp) f(e, m)).

        L: (Np, M) float32; f: (E, M) for "em", (M, E) for "dm"; sc: (E, nf)
        for "em", (nf, E) for "dm"; M = nf * nfp."""
        L_, pL = _f32(L)
        Np, M = L_.shape
        assert M % nf == 0
        nfp = M // nf
        f_, pf = _f32(f)
        s_, ps = _f32(sc)
        E = f_.shape[0] if layout == "em" else f_.shape[1]
        assert f_.shape == ((E, M) if layout == "em" else (M, E))
        assert s_.shape == ((E, nf) if layout == "em" else (nf, E))
        if ne is None:
            ne = E - e0
        assert 0 <= e0 and e0 + ne <= E
        ref = np.zeros((ne, Np), dtype=np.float64)
        self.L.oracle_dg_surface(Np, nf, nfp, E, LAYOUT[layout], PREC[precision], pL, pf, ps,
                                 e0, ne, ref.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return ref

    def coulomb(self, targets, sources, layout="em", t0=0, n=None):
        """FP64 potential ref[t - t0] = sum_s q_s / |x_t - y_s| (pairs at zero
        distance skipped).  layout "em" (AoS): targets (nt, 4) with columns
        x, y, z, unused; sources (ns, 4) = x, y, z, q.  "dm" (SoA): targets
        (3, nt), sources (4, ns)."""
        tg, pt = _f32(targets)
        sr, ps = _f32(sources)
        if layout == "em":
            assert tg.ndim == 2 and tg.shape[1] == 4 and sr.ndim == 2 and sr.shape[1] == 4
            nt, ns = tg.shape[0], sr.shape[0]
        else:
            assert tg.ndim == 2 and tg.shape[0] == 3 and sr.ndim == 2 and sr.shape[0] == 4
            nt, ns = tg.shape[1], sr.shape[1]
        if n is None:
            n = nt - t0
        assert 0 <= t0 and t0 + n <= nt
        ref = np.zeros(n, dtype=np.float64)
        self.L.oracle_coulomb(nt, ns, LAYOUT[layout], pt, ps, t0, n,
                              ref.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return ref

    def gemm(self, A, B, precision="fp32", m0=0, nm=None):
        """FP64 reference rows C[m0:m0+nm, :] of C = A @ B (row-major)."""
        A, pA = _f32(A)
        B, pB = _f32(B)
        M, Kd = A.shape
        Kd2, N = B.shape
        assert Kd == Kd2
        if nm is None:
            nm = M - m0
        C = np.zeros((nm, N), dtype=np.float64)
        self.L.oracle_gemm(M, N, Kd, PREC[precision], pA, pB, m0, nm,
                           C.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return C


_default = None


def default() -> Oracle:
    """The oracle built from ``oracle.c`` (built on first use if absent)."""
    global _default
    if _default is None:
        if not os.path.exists(LIB):
            build()
        _default = Oracle(LIB)
    return _default


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def threads() -> int:
    return default().threads()


def set_threads(n: int) -> None:
    default().set_threads(n)


def bf16_rne(x):
    return default().bf16_rne(x)


def split_bf16(x):
    return default().split_bf16(x)


def contract(D, u, layout="em", precision="fp32", e0=0, ne=None):
    return default().contract(D, u, layout, precision, e0, ne)


def gemm(A, B, precision="fp32", m0=0, nm=None):
    return default().gemm(A, B, precision, m0, nm)


def dg_surface(L, f, sc, nf, layout="em", precision="fp32", e0=0, ne=None):
    return default().dg_surface(L, f, sc, nf, layout, precision, e0, ne)


def coulomb(targets, sources, layout="em", t0=0, n=None):
    return default().coulomb(targets, sources, layout, t0, n)


def dg_volume(D, u, G, layout="em", precision="fp32", e0=0, ne=None):
    return default().dg_volume(D, u, G, layout, precision, e0, ne)


def rel_err(y, ref) -> float:
    """Normwise relative error max|y - ref| / max|ref| (inf-norm)."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(y - ref))) if ref.size else 0.0
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den
