"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the
oracle's tests.  This module holds random-number draws and shapes only, none
of the method's arithmetic.

Generator: numpy PCG64 (``default_rng(seed)``), arrays drawn in the order
D then u (or A then B), cast to float32.  N(0, s^2) means standard deviation
s.  The workloads mirror the paper's Table 1 kinds ("dG FEM volume",
"sgemm"); the paper gives no sizes, so these synthetic shapes stand in.
"""
import math

import numpy as np

# Operator orders of the ragged-batch workload: the node counts of
# tetrahedral elements of degree 2..7.
RAGGED_NP = (10, 20, 35, 56, 84, 120)


def _uniform(rng, shape, lo=-1.0, hi=1.0):
    return rng.uniform(lo, hi, size=shape).astype(np.float32)


def contraction_inputs(K, Np, E, seed=0, layout="em"):
    """D ~ N(0, 1/Np) of shape (K, Np, Np); u ~ U(-1, 1) of shape (E, Np)
    for element-major, or the same values stored (Np, E) for DOF-major."""
    rng = np.random.default_rng(seed)
    D = rng.normal(0.0, 1.0 / math.sqrt(Np), size=(K, Np, Np)).astype(np.float32)
    u = _uniform(rng, (E, Np))
    if layout == "dm":
        u = np.ascontiguousarray(u.T)
    return D, u


def dg_volume_inputs(K, Np, E, seed=0, layout="em"):
    """(D, u, G) for the dG volume workload: D and u exactly as
    contraction_inputs draws them for the same seed, then per-element
    geometric factors G[e] = s_e (I + 0.25 N(0, 1)^{K x K}) with the element
    scale s_e ~ U(0.5, 2) (an affine element's inverse Jacobian: near a
    scaled identity, well conditioned, sizes varying across the mesh).
    G has shape (E, K, K) for element-major, the same values stored
    (K, K, E) for DOF-major."""
    rng = np.random.default_rng(seed)
    D = rng.normal(0.0, 1.0 / math.sqrt(Np), size=(K, Np, Np)).astype(np.float32)
    u = _uniform(rng, (E, Np))
    s = rng.uniform(0.5, 2.0, size=(E, 1, 1))
    G = (s * (np.eye(K)[None] + 0.25 * rng.standard_normal((E, K, K)))).astype(np.float32)
    if layout == "dm":
        u = np.ascontiguousarray(u.T)
        G = np.ascontiguousarray(G.transpose(1, 2, 0))
    return D, u, G


def dg_surface_inputs(Np, nf, nfp, E, seed=0, layout="em"):
    """(L, f, s) for the dG surface (lift) workload: L ~ N(0, 1/M) of shape
    (Np, M), M = nf * nfp; face fluxes f ~ U(-1, 1); per-face factors
    s ~ U(0.5, 2) (surface-to-volume Jacobian ratios), drawn in that order.
    Element-major: f (E, M), s (E, nf); DOF-major: the same values stored
    (M, E) and (nf, E)."""
    rng = np.random.default_rng(seed)
    M = nf * nfp
    L = rng.normal(0.0, 1.0 / math.sqrt(M), size=(Np, M)).astype(np.float32)
    f = _uniform(rng, (E, M))
    s = rng.uniform(0.5, 2.0, size=(E, nf)).astype(np.float32)
    if layout == "dm":
        f = np.ascontiguousarray(f.T)
        s = np.ascontiguousarray(s.T)
    return L, f, s


def coulomb_inputs(nt, ns, seed=0, layout="em"):
    """Targets and point charges for the Coulomb potential: target and
    source positions uniform in the unit cube, charges q ~ U(-1, 1), drawn
    in that order.  Element-major ("em", array of structures): targets
    (nt, 4) = x, y, z, 0 and sources (ns, 4) = x, y, z, q; DOF-major ("dm",
    structure of arrays): targets (3, nt), sources (4, ns)."""
    rng = np.random.default_rng(seed)
    xt = rng.uniform(0.0, 1.0, size=(nt, 3)).astype(np.float32)
    xs = rng.uniform(0.0, 1.0, size=(ns, 3)).astype(np.float32)
    q = _uniform(rng, (ns,))
    if layout == "em":
        tg = np.zeros((nt, 4), np.float32)
        tg[:, :3] = xt
        sr = np.concatenate([xs, q[:, None]], axis=1).astype(np.float32)
        return tg, np.ascontiguousarray(sr)
    return np.ascontiguousarray(xt.T), np.ascontiguousarray(np.concatenate([xs.T, q[None]]))


def integer_contraction_inputs(K, Np, E, seed=0, layout="em", bound=8):
    """Small-integer operands in [-bound, bound]: every product and partial
    sum is exact in FP32 (and in bf16 for |x| <= 256)."""
    rng = np.random.default_rng(seed)
    D = rng.integers(-bound, bound + 1, size=(K, Np, Np)).astype(np.float32)
    u = rng.integers(-bound, bound + 1, size=(E, Np)).astype(np.float32)
    if layout == "dm":
        u = np.ascontiguousarray(u.T)
    return D, u


def gemm_inputs(M, N, K, seed=0):
    """A ~ N(0,1) of shape (M, K), B ~ N(0,1) of shape (K, N), float32."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((M, K), dtype=np.float32)
    B = rng.standard_normal((K, N), dtype=np.float32)
    return A, B


def integer_gemm_inputs(M, N, K, seed=0, bound=4):
    rng = np.random.default_rng(seed)
    A = rng.integers(-bound, bound + 1, size=(M, K)).astype(np.float32)
    B = rng.integers(-bound, bound + 1, size=(K, N)).astype(np.float32)
    return A, B


def ragged_shapes(n=512, seed=0, lo=1024, hi=65536):
    """(Np, E) per instance: Np uniform over RAGGED_NP, E log-uniform in
    [lo, hi] (E = floor(exp(U(ln lo, ln hi))))."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        Np = int(RAGGED_NP[int(rng.integers(0, len(RAGGED_NP)))])
        E = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        out.append((Np, E))
    return out


def ragged_batch_inputs(shapes, K=3, seed=0):
    """One (D, u) pair per instance, element-major, drawn in instance order
    from a single generator: D ~ N(0, 1/Np), u ~ U(-1, 1)."""
    rng = np.random.default_rng(seed + 1)
    items = []
    for Np, E in shapes:
        D = rng.normal(0.0, 1.0 / math.sqrt(Np), size=(K, Np, Np)).astype(np.float32)
        u = _uniform(rng, (E, Np))
        items.append((D, u))
    return items


def picker_shapes(n, seed, precisions=("fp32", "bf16x3", "bf16")):
    """Random problem shapes for cost-model training/evaluation:
    Np uniform integer in [8, 128], E = floor(2^U(10, 21)), each rounded up
    (Np) or down (E) to a multiple of 4 with probability 1/2, so that the
    four 16-byte alignment classes of rows and element runs are equally
    common; layout and precision uniform, K = 3."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        Np = int(rng.integers(8, 129))
        if rng.random() < 0.5:
            Np = 4 * ((Np + 3) // 4)
        E = int(math.floor(2.0 ** rng.uniform(10.0, 21.0)))
        if rng.random() < 0.5:
            E = 4 * (E // 4)
        layout = ("em", "dm")[int(rng.integers(0, 2))]
        prec = precisions[int(rng.integers(0, len(precisions)))]
        out.append({"K": 3, "Np": Np, "E": E, "layout": layout, "precision": prec})
    return out
