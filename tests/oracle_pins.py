"""Pins of the FP64 oracle against facts fixed by the mathematics and by
independent library routines, not by the oracle itself.

Each pin takes an ``oracle.Oracle`` handle, so the same checks run against
the real oracle (must pass) and against deliberately mutated builds of it
(each mutant must fail at least one pin).  The contraction is the reduction
sum(j, D[k,i,j]*u[e,j]) of the paper's sec. 2.1; GEMM is its sum(k,
a[i,k]*b[k,j]) example.
"""
from fractions import Fraction

import numpy as np
import torch

from paper_1405_7470_amd import inputs


def _bf16_lib(x):
    """bfloat16 rounding by torch (round-to-nearest-even), an independent
    library routine, returned as float32."""
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float32).numpy()


def _operands(x, precision):
    """Operand pieces per precision mode, rounded by the library routine."""
    x = np.asarray(x, dtype=np.float32)
    if precision == "fp32":
        return x, None
    hi = _bf16_lib(x)
    if precision == "bf16":
        return hi, None
    lo = _bf16_lib((x - hi).astype(np.float32))  # exact FP32 subtraction
    return hi, lo


def _exact_contract(D, u, layout, precision):
    """Exact rational value of the contraction under a precision mode."""
    K, Np, _ = D.shape
    E = u.shape[0] if layout == "em" else u.shape[1]
    ue = u if layout == "em" else u.T
    Dh, Dl = _operands(D, precision)
    uh, ul = _operands(ue, precision)
    out = np.empty((K, E, Np), dtype=object)
    for k in range(K):
        for e in range(E):
            for i in range(Np):
                s = Fraction(0)
                for j in range(Np):
                    s += Fraction(float(Dh[k, i, j])) * Fraction(float(uh[e, j]))
                    if precision == "bf16x3":
                        s += Fraction(float(Dh[k, i, j])) * Fraction(float(ul[e, j]))
                        s += Fraction(float(Dl[k, i, j])) * Fraction(float(uh[e, j]))
                out[k, e, i] = s
    return out


def _assert_close_exact(ref, exact, Np):
    """FP64 accumulation of exact products: error <= Np * 2^-52 * sum|terms|,
    bounded here by Np * 2^-52 * (max|exact| + slack) using term magnitudes."""
    diff = max(abs(Fraction(float(r)) - x) for r, x in zip(ref.ravel(), exact.ravel()))
    scale = max(abs(x) for x in exact.ravel()) + 1
    assert diff <= Fraction(Np * 4) * Fraction(2) ** -52 * scale * 16, float(diff)


def pin_contract_bruteforce(o):
    """Tiny random shapes, every precision and layout, against exact rational
    sums (FP32 products are exact in FP64, so only FP64 rounding remains)."""
    rng = np.random.default_rng(11)
    for (K, Np, E) in [(1, 1, 1), (2, 3, 5), (3, 5, 7), (2, 4, 3)]:
        D = rng.normal(0, 1, (K, Np, Np)).astype(np.float32)
        u = rng.uniform(-1, 1, (E, Np)).astype(np.float32)
        for precision in ("fp32", "bf16", "bf16x3"):
            exact = _exact_contract(D, u, "em", precision)
            for layout in ("em", "dm"):
                uu = u if layout == "em" else np.ascontiguousarray(u.T)
                ref = o.contract(D, uu, layout, precision)
                _assert_close_exact(ref, exact, Np)


def pin_contract_identity(o):
    """D_k = I gives out = u exactly (both layouts)."""
    K, Np, E = 3, 7, 33
    _, u = inputs.contraction_inputs(K, Np, E, seed=3)
    D = np.stack([np.eye(Np, dtype=np.float32)] * K)
    for layout in ("em", "dm"):
        uu = u if layout == "em" else np.ascontiguousarray(u.T)
        ref = o.contract(D, uu, layout, "fp32")
        for k in range(K):
            assert np.array_equal(ref[k], u.astype(np.float64))


def pin_contract_ones(o):
    """All-ones D gives every output row the sum of the element's values;
    a permuted identity picks out one column."""
    K, Np, E = 2, 6, 19
    rng = np.random.default_rng(5)
    u = rng.integers(-50, 51, (E, Np)).astype(np.float32)
    D = np.ones((K, Np, Np), dtype=np.float32)
    ref = o.contract(D, u, "em", "fp32")
    rows = u.astype(np.float64).sum(axis=1)
    for k in range(K):
        for i in range(Np):
            assert np.array_equal(ref[k, :, i], rows)
    perm = rng.permutation(Np)
    P = np.zeros((1, Np, Np), dtype=np.float32)
    P[0, np.arange(Np), perm] = 1.0          # row i picks column perm[i]
    ref = o.contract(P, u, "em", "fp32")
    assert np.array_equal(ref[0], u[:, perm].astype(np.float64))


def pin_contract_rank1(o):
    """u(e, j) = a_e b_j gives out(k, e, i) = a_e (D_k b)_i (integers, exact)."""
    rng = np.random.default_rng(9)
    K, Np, E = 2, 9, 12
    a = rng.integers(-6, 7, E).astype(np.float64)
    b = rng.integers(-6, 7, Np).astype(np.float64)
    D = rng.integers(-5, 6, (K, Np, Np)).astype(np.float32)
    u = np.outer(a, b).astype(np.float32)
    ref = o.contract(D, u, "em", "fp32")
    for k in range(K):
        Db = np.array([sum(float(D[k, i, j]) * b[j] for j in range(Np)) for i in range(Np)])
        assert np.array_equal(ref[k], np.outer(a, Db))


def pin_contract_zero_and_linearity(o):
    K, Np, E = 2, 8, 21
    rng = np.random.default_rng(13)
    D = rng.integers(-7, 8, (K, Np, Np)).astype(np.float32)
    u = rng.integers(-7, 8, (E, Np)).astype(np.float32)
    v = rng.integers(-7, 8, (E, Np)).astype(np.float32)
    assert not np.any(o.contract(np.zeros_like(D), u, "em", "fp32"))
    lhs = o.contract(D, (3 * u - 2 * v).astype(np.float32), "em", "fp32")
    rhs = 3 * o.contract(D, u, "em", "fp32") - 2 * o.contract(D, v, "em", "fp32")
    assert np.array_equal(lhs, rhs)


def pin_contract_layouts_and_chunks(o):
    """Element-major and DOF-major storage of the same values give the same
    result; chunked evaluation equals the whole."""
    K, Np, E = 3, 11, 40
    D, u = inputs.contraction_inputs(K, Np, E, seed=21)
    a = o.contract(D, u, "em", "fp32")
    b = o.contract(D, np.ascontiguousarray(u.T), "dm", "fp32")
    assert np.array_equal(a, b)
    parts = [o.contract(D, u, "em", "fp32", e0, n) for e0, n in ((0, 13), (13, 1), (14, 26))]
    assert np.array_equal(np.concatenate(parts, axis=1), a)


def pin_contract_integer_all_precisions(o):
    """Integer operands |x| <= 8 are exact in bf16, so every precision mode
    gives the exact integer result (lo parts vanish)."""
    K, Np, E = 3, 10, 25
    D, u = inputs.integer_contraction_inputs(K, Np, E, seed=4)
    exact = np.einsum("kij,ej->kei", D.astype(np.int64), u.astype(np.int64))
    for precision in ("fp32", "bf16", "bf16x3"):
        assert np.array_equal(o.contract(D, u, "em", precision), exact.astype(np.float64))


def pin_bf16_rounding(o):
    """bf16 rounding agrees with torch's round-to-nearest-even conversion on
    random values over many binades and on special values."""
    rng = np.random.default_rng(17)
    x = (rng.standard_normal(200000) * np.exp2(rng.integers(-130, 120, 200000))).astype(np.float32)
    base = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)
    specials = np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, -3.0e38, 3.3895314e38, 1e-40, -1e-40,
                         np.inf, -np.inf,
                         base + ulp / 2, base + 3 * ulp / 2, base + ulp / 2 + 2.0 ** -20,
                         -(base + ulp / 2), 2.0 ** -126, 2.0 ** -133 * 3],
                        dtype=np.float32)
    for arr in (x, specials):
        mine = o.bf16_rne(arr)
        lib = _bf16_lib(arr)
        assert np.array_equal(mine.view(np.uint32), lib.view(np.uint32))
    nan = o.bf16_rne(np.array([np.nan], dtype=np.float32))
    assert np.isnan(nan[0])
    # ties go to even: 1 + 2^-8 -> 1 ; 1 + 3*2^-8 -> 1 + 2^-6
    t = o.bf16_rne(np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8], dtype=np.float32))
    assert t[0] == 1.0 and t[1] == 1 + 2 ** -6


def pin_split_bf16(o):
    """hi and lo are bf16 values; x - hi is exact in FP32 and hi + lo
    approximates x to 2^-16 relative."""
    rng = np.random.default_rng(19)
    x = rng.standard_normal(100000).astype(np.float32)
    hi, lo = o.split_bf16(x)
    assert not np.any(hi.view(np.uint32) & 0xFFFF)
    assert not np.any(lo.view(np.uint32) & 0xFFFF)
    assert np.array_equal(hi, _bf16_lib(x))
    assert np.array_equal(lo, _bf16_lib((x - hi).astype(np.float32)))
    err = np.abs(x.astype(np.float64) - hi - lo)
    assert np.all(err <= 2.0 ** -16 * np.abs(x))


def pin_precision_error_bands(o):
    """Reduced-precision modes sit in their error bands against the exact
    FP32-operand sum: bf16 ~1e-3 (8-bit operands), bf16x3 ~1e-6..1e-5."""
    K, Np, E = 3, 56, 3000
    D, u = inputs.contraction_inputs(K, Np, E, seed=23)
    r32 = o.contract(D, u, "em", "fp32")
    den = np.max(np.abs(r32))
    e1 = np.max(np.abs(o.contract(D, u, "em", "bf16") - r32)) / den
    e3 = np.max(np.abs(o.contract(D, u, "em", "bf16x3") - r32)) / den
    assert 1e-4 < e1 < 2e-2, e1
    assert 1e-7 < e3 < 1e-5, e3


def pin_gemm(o):
    rng = np.random.default_rng(29)
    # tiny: exact rational sums
    A = rng.normal(0, 1, (3, 5)).astype(np.float32)
    B = rng.normal(0, 1, (5, 4)).astype(np.float32)
    C = o.gemm(A, B)
    for m in range(3):
        for n in range(4):
            ex = sum(Fraction(float(A[m, k])) * Fraction(float(B[k, n])) for k in range(5))
            assert abs(Fraction(float(C[m, n])) - ex) <= Fraction(2) ** -48 * (abs(ex) + 1)
    # numpy float64 matmul (library routine) on a non-square case
    A, B = inputs.gemm_inputs(37, 53, 71, seed=2)
    C = o.gemm(A, B)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    assert np.max(np.abs(C - ref)) <= 1e-12 * np.max(np.abs(ref))
    # identity and integer exactness
    I = np.eye(53, dtype=np.float32)
    Bs = np.ascontiguousarray(B[:53])
    assert np.array_equal(o.gemm(I, Bs), Bs.astype(np.float64))
    Ai, Bi = inputs.integer_gemm_inputs(19, 23, 31, seed=6)
    exact = Ai.astype(np.int64) @ Bi.astype(np.int64)
    for precision in ("fp32", "bf16", "bf16x3"):
        assert np.array_equal(o.gemm(Ai, Bi, precision), exact.astype(np.float64))
    # row chunks
    full = o.gemm(A, B)
    assert np.array_equal(np.concatenate([o.gemm(A, B, "fp32", 0, 10), o.gemm(A, B, "fp32", 10, 27)]), full)
    # bf16x3 error band on a GEMM
    A, B = inputs.gemm_inputs(64, 64, 512, seed=8)
    r = o.gemm(A, B)
    e3 = np.max(np.abs(o.gemm(A, B, "bf16x3") - r)) / np.max(np.abs(r))
    assert 1e-8 < e3 < 1e-5, e3


def _g_as_em(G, layout):
    return G if layout == "em" else np.ascontiguousarray(G.transpose(2, 0, 1))


def _g_store(G_em, layout):
    return G_em if layout == "em" else np.ascontiguousarray(G_em.transpose(1, 2, 0))


def pin_dg_bruteforce(o):
    """dG volume on tiny shapes against exact rational sums: the exact
    contraction (per precision) combined with the exact geometric factors."""
    rng = np.random.default_rng(21)
    for (K, Np, E) in [(1, 1, 1), (2, 3, 4), (3, 4, 5), (3, 2, 3)]:
        D = rng.normal(0, 1, (K, Np, Np)).astype(np.float32)
        u = rng.uniform(-1, 1, (E, Np)).astype(np.float32)
        G = rng.normal(0, 1, (E, K, K)).astype(np.float32)
        for precision in ("fp32", "bf16x3"):
            c = _exact_contract(D, u, "em", precision)
            exact = np.empty((K, E, Np), dtype=object)
            for d in range(K):
                for e in range(E):
                    for i in range(Np):
                        exact[d, e, i] = sum(Fraction(float(G[e, d, k])) * c[k, e, i]
                                             for k in range(K))
            for layout in ("em", "dm"):
                uu = u if layout == "em" else np.ascontiguousarray(u.T)
                ref = o.dg_volume(D, uu, _g_store(G, layout), layout, precision)
                _assert_close_exact(ref, exact, Np * K)


def pin_dg_identity_and_diagonal(o):
    """G = I gives the contraction itself, bit for bit; a diagonal G of
    signed powers of two scales each reference derivative exactly."""
    K, Np, E = 3, 20, 37
    D, u, _ = inputs.dg_volume_inputs(K, Np, E, seed=3)
    rng = np.random.default_rng(4)
    for layout in ("em", "dm"):
        uu = u if layout == "em" else np.ascontiguousarray(u.T)
        c = o.contract(D, uu, layout, "fp32")
        I = np.broadcast_to(np.eye(K, dtype=np.float32), (E, K, K)).copy()
        assert np.array_equal(o.dg_volume(D, uu, _g_store(I, layout), layout), c)
        sc = (rng.choice([-1.0, 1.0], (E, K)) * 2.0 ** rng.integers(-3, 4, (E, K)))
        Gd = np.zeros((E, K, K), np.float32)
        for d in range(K):
            Gd[:, d, d] = sc[:, d]
        ref = o.dg_volume(D, uu, _g_store(Gd, layout), layout)
        assert np.array_equal(ref, c * sc.T[:, :, None])


def pin_dg_permutation_and_linearity(o):
    """A permutation metric picks reference derivatives (exactly); the result
    is linear in G (to FP64 rounding)."""
    K, Np, E = 3, 12, 29
    D, u, G1 = inputs.dg_volume_inputs(K, Np, E, seed=5)
    _, _, G2 = inputs.dg_volume_inputs(K, Np, E, seed=6)
    c = o.contract(D, u, "em", "fp32")
    perm = [2, 0, 1]
    P = np.zeros((E, K, K), np.float32)
    for d in range(K):
        P[:, d, perm[d]] = 1.0
    assert np.array_equal(o.dg_volume(D, u, P), c[perm])
    # element-varying permutations
    Pe = np.zeros((E, K, K), np.float32)
    for e in range(E):
        pe = np.roll(np.arange(K), e)
        for d in range(K):
            Pe[e, d, pe[d]] = 1.0
    ref = o.dg_volume(D, u, Pe)
    for e in range(E):
        pe = np.roll(np.arange(K), e)
        assert np.array_equal(ref[:, e], c[pe, e])
    a = o.dg_volume(D, u, G1) + o.dg_volume(D, u, G2)
    b = o.dg_volume(D, u, (G1 + G2).astype(np.float32))
    # G1 + G2 rounded to float32: compare against the exactly summed factors
    assert np.max(np.abs(a - b)) <= 1e-6 * np.max(np.abs(a))


def pin_dg_layouts_chunks_integers(o):
    """Element-major and DOF-major storage give the same values; chunks equal
    the whole; small-integer inputs are exact in every precision."""
    K, Np, E = 3, 16, 53
    D, u, G = inputs.dg_volume_inputs(K, Np, E, seed=7)
    em = o.dg_volume(D, u, G, "em")
    dm = o.dg_volume(D, np.ascontiguousarray(u.T), _g_store(G, "dm"), "dm")
    assert np.array_equal(em, dm)
    assert np.array_equal(o.dg_volume(D, u, G, "em", "fp32", 10, 20), em[:, 10:30])
    Di, ui = inputs.integer_contraction_inputs(K, Np, E, seed=8, bound=4)
    Gi = np.random.default_rng(9).integers(-3, 4, (E, K, K)).astype(np.float32)
    exact = np.einsum("edk,kij,ej->dei", Gi.astype(np.int64), Di.astype(np.int64),
                      ui.astype(np.int64)).astype(np.float64)
    for precision in ("fp32", "bf16", "bf16x3"):
        assert np.array_equal(o.dg_volume(Di, ui, Gi, "em", precision), exact)


def pin_dg_surface_bruteforce(o):
    """The lift on tiny shapes against exact rational sums of the FP32-
    rounded scaled fluxes (numpy's float32 product) times the operator,
    operands rounded per precision by the library bf16 routine."""
    rng = np.random.default_rng(41)
    for (Np, nf, nfp, E) in [(1, 1, 1, 1), (3, 2, 2, 4), (5, 4, 3, 3), (4, 3, 1, 2)]:
        M = nf * nfp
        L = rng.normal(0, 1, (Np, M)).astype(np.float32)
        f = rng.uniform(-1, 1, (E, M)).astype(np.float32)
        sc = rng.uniform(0.5, 2, (E, nf)).astype(np.float32)
        g = (np.repeat(sc, nfp, axis=1) * f).astype(np.float32)
        for precision in ("fp32", "bf16", "bf16x3"):
            Lh, Ll = _operands(L, precision)
            gh, gl = _operands(g, precision)
            exact = np.empty((E, Np), dtype=object)
            for e in range(E):
                for i in range(Np):
                    t = Fraction(0)
                    for m in range(M):
                        t += Fraction(float(Lh[i, m])) * Fraction(float(gh[e, m]))
                        if precision == "bf16x3":
                            t += Fraction(float(Lh[i, m])) * Fraction(float(gl[e, m]))
                            t += Fraction(float(Ll[i, m])) * Fraction(float(gh[e, m]))
                    exact[e, i] = t
            for layout in ("em", "dm"):
                ff = f if layout == "em" else np.ascontiguousarray(f.T)
                ss = sc if layout == "em" else np.ascontiguousarray(sc.T)
                ref = o.dg_surface(L, ff, ss, nf, layout, precision)
                _assert_close_exact(ref, exact, M)


def pin_dg_surface_against_contraction(o):
    """One face (nf = 1) with unit factors and a square operator is the
    contraction with K = 1, bit for bit; a factor of 2^k on a face scales
    exactly the part of the sum that face contributes."""
    Np, E = 12, 17
    D, u = inputs.contraction_inputs(1, Np, E, seed=9)
    for precision in ("fp32", "bf16x3"):
        ref = o.dg_surface(D[0], u, np.ones((E, 1), np.float32), 1, "em", precision)
        assert np.array_equal(ref, o.contract(D, u, "em", precision)[0])
    # two faces of nfp = 6: face 1's factor 4, face 0's 1 -> contraction of the
    # face-0 half plus 4x the contraction of the face-1 half
    L, f, _ = inputs.dg_surface_inputs(Np, 2, 6, E, seed=10)
    sc = np.ones((E, 2), np.float32)
    sc[:, 1] = 4.0
    got = o.dg_surface(L, f, sc, 2)
    h0 = o.dg_surface(L[:, :6].copy(), f[:, :6].copy(), np.ones((E, 1), np.float32), 1)
    h1 = o.dg_surface(L[:, 6:].copy(), f[:, 6:].copy(), np.ones((E, 1), np.float32), 1)
    assert np.max(np.abs(got - (h0 + 4 * h1))) <= 1e-14 * np.max(np.abs(got))


def pin_dg_surface_layouts_chunks_integers(o):
    Np, nf, nfp, E = 10, 4, 5, 23
    L, f, sc = inputs.dg_surface_inputs(Np, nf, nfp, E, seed=11)
    em = o.dg_surface(L, f, sc, nf, "em")
    dm = o.dg_surface(L, np.ascontiguousarray(f.T), np.ascontiguousarray(sc.T), nf, "dm")
    assert np.array_equal(em, dm)
    assert np.array_equal(o.dg_surface(L, f, sc, nf, "em", "fp32", 5, 9), em[5:14])
    rng = np.random.default_rng(12)
    Li = rng.integers(-4, 5, (Np, nf * nfp)).astype(np.float32)
    fi = rng.integers(-4, 5, (E, nf * nfp)).astype(np.float32)
    si = (2.0 ** rng.integers(-2, 3, (E, nf))).astype(np.float32)
    exact = (np.repeat(si, nfp, axis=1).astype(np.float64) * fi) @ Li.T.astype(np.float64)
    for precision in ("fp32", "bf16", "bf16x3"):
        assert np.array_equal(o.dg_surface(Li, fi, si, nf, "em", precision), exact)


def _coulomb_aos(xt, xs, q):
    tg = np.zeros((len(xt), 4), np.float32)
    tg[:, :3] = xt
    sr = np.zeros((len(xs), 4), np.float32)
    sr[:, :3] = xs
    sr[:, 3] = q
    return tg, sr


def pin_coulomb_closed_forms(o):
    """A single charge at Pythagorean offsets (3-4-12-13 and 2-3-6-7 triples,
    square roots exact) and a target at the centre of a cube of eight equal
    charges: the potential q / r of the mathematics."""
    xs = np.array([[0.5, 0.25, 0.125]], np.float32)
    q = np.array([0.75], np.float32)
    xt = xs + np.array([[3, 4, 12], [2, 3, 6], [-6, 2, -3], [0, 0, 2]], np.float32)
    tg, sr = _coulomb_aos(xt, xs, q)
    ref = o.coulomb(tg, sr)
    assert list(ref) == [0.75 / 13.0, 0.75 / 7.0, 0.75 / 7.0, 0.375]
    a = 0.5
    corners = np.array([[sx * a, sy * a, sz * a] for sx in (-1, 1) for sy in (-1, 1)
                        for sz in (-1, 1)], np.float32)
    tg, sr = _coulomb_aos(np.zeros((1, 3), np.float32), corners, np.full(8, 2.0, np.float32))
    want = 8 * 2.0 / (a * np.sqrt(3.0))
    assert abs(o.coulomb(tg, sr)[0] - want) <= 1e-15 * want


def pin_coulomb_bruteforce_and_self_pairs(o):
    """Small random sets against a numpy FP64 pairwise sum; targets equal to
    the sources: the zero-distance pair of each target contributes nothing."""
    rng = np.random.default_rng(31)
    xt = rng.uniform(0, 1, (50, 3)).astype(np.float32)
    xs = rng.uniform(0, 1, (70, 3)).astype(np.float32)
    q = rng.uniform(-1, 1, 70).astype(np.float32)
    for a, b in ((xt, xs), (xs, xs)):
        tg, sr = _coulomb_aos(a, b, q)
        d = a.astype(np.float64)[:, None, :] - b.astype(np.float64)[None, :, :]
        r = np.sqrt((d * d).sum(-1))
        with np.errstate(divide="ignore"):
            w = np.where(r > 0, q.astype(np.float64)[None, :] / r, 0.0)
        want = w.sum(1)
        got = o.coulomb(tg, sr)
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def pin_coulomb_scaling_and_superposition(o):
    """Doubling every coordinate halves the potential exactly (power-of-two
    scaling commutes with rounding); charges add (dyadic charges, so their
    FP32 sum is exact)."""
    tg, sr = inputs.coulomb_inputs(40, 90, seed=3)
    ref = o.coulomb(tg, sr)
    tg2, sr2 = tg.copy(), sr.copy()
    tg2[:, :3] *= 2
    sr2[:, :3] *= 2
    assert np.array_equal(o.coulomb(tg2, sr2), ref / 2)
    rng = np.random.default_rng(4)
    q1 = rng.integers(-8, 9, 90).astype(np.float32) / 8
    q2 = rng.integers(-8, 9, 90).astype(np.float32) / 8
    sa, sb, sc = sr.copy(), sr.copy(), sr.copy()
    sa[:, 3], sb[:, 3], sc[:, 3] = q1, q2, q1 + q2
    s = o.coulomb(tg, sa) + o.coulomb(tg, sb)
    assert np.max(np.abs(o.coulomb(tg, sc) - s)) <= 1e-13 * np.max(np.abs(s))


def pin_coulomb_layouts_chunks(o):
    """Array-of-structures and structure-of-arrays storage give the same
    values; a chunk of targets equals the same rows of the whole."""
    tg, sr = inputs.coulomb_inputs(33, 57, seed=5, layout="em")
    tgd, srd = inputs.coulomb_inputs(33, 57, seed=5, layout="dm")
    assert np.array_equal(tgd, tg[:, :3].T) and np.array_equal(srd, sr.T)
    em = o.coulomb(tg, sr, "em")
    assert np.array_equal(o.coulomb(tgd, srd, "dm"), em)
    assert np.array_equal(o.coulomb(tg, sr, "em", 7, 11), em[7:18])
    assert np.array_equal(o.coulomb(tgd, srd, "dm", 20, 13), em[20:33])


ALL_PINS = [
    pin_contract_bruteforce,
    pin_contract_identity,
    pin_contract_ones,
    pin_contract_rank1,
    pin_contract_zero_and_linearity,
    pin_contract_layouts_and_chunks,
    pin_contract_integer_all_precisions,
    pin_bf16_rounding,
    pin_split_bf16,
    pin_precision_error_bands,
    pin_gemm,
    pin_dg_bruteforce, pin_dg_identity_and_diagonal, pin_dg_permutation_and_linearity,
    pin_dg_layouts_chunks_integers,
    pin_coulomb_closed_forms, pin_coulomb_bruteforce_and_self_pairs,
    pin_coulomb_scaling_and_superposition, pin_coulomb_layouts_chunks,
    pin_dg_surface_bruteforce, pin_dg_surface_against_contraction,
    pin_dg_surface_layouts_chunks_integers,
]
