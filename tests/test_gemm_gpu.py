"""GEMM (the contraction's degenerate case) through lpx_gemm vs the FP64
oracle: every built tiling and precision on ragged shapes, exact integer
inputs, identity, K = 0, and at 4096^3 and 8192 x 1024 x 4096 a NaN sentinel
over all of C plus one row of every m-tile and a column stripe of every
n-tile."""
import numpy as np
import pytest
import torch

import oracle
from paper_1405_7470_amd import inputs, lpx
from tests.gpu_util import SHORT_REDUCTION, TOL, assert_within_bound, emu_tol, to_dev

pytestmark = pytest.mark.gpu

TILES = {"fp32": [(64, 64, 32), (64, 64, 64), (128, 128, 32), (128, 128, 64), (128, 64, 32),
                  (64, 128, 32), (256, 128, 32), (128, 256, 32), (256, 256, 32)],
         "bf16": [(64, 64, 32), (128, 128, 32), (128, 128, 64), (256, 256, 32), (256, 256, 64),
                  (256, 128, 64)],
         "bf16x3": [(64, 64, 32), (64, 64, 64), (128, 128, 32), (128, 128, 64), (64, 128, 32),
                    (256, 256, 32), (256, 128, 32)]}
# tilings that run the pre-split kernel (operands split into bf16 planes first)
PRESPLIT = {"bf16": [(128, 128, 64), (256, 256, 64), (256, 128, 64)],
            "bf16x3": [(128, 128, 64), (256, 256, 32), (256, 128, 32)]}


def check(C, A, B, precision, m0=0):
    nm = C.shape[0]
    ref = oracle.gemm(A, B, "fp32", m0, nm)
    err = oracle.rel_err(C, ref)
    if precision == "bf16x3" and A.shape[1] < SHORT_REDUCTION:
        absref = oracle.gemm(np.abs(A), np.abs(B), "fp32", m0, nm)
        assert_within_bound(C, ref, absref, A.shape[1], precision)
    else:
        assert err <= TOL[precision], (precision, err)
    if precision != "fp32":
        emu = oracle.gemm(A, B, precision, m0, nm)
        assert oracle.rel_err(C, emu) <= emu_tol(A.shape[1])
    return err


@pytest.mark.parametrize("precision", ("fp32", "bf16", "bf16x3"))
def test_gemm_tilings_ragged(precision):
    for (M, N, K) in ((128, 128, 128), (100, 77, 61), (257, 130, 95), (33, 300, 1)):
        A, B = inputs.gemm_inputs(M, N, K, seed=M + N + K)
        Ad, Bd = to_dev(A), to_dev(B)
        for tiles in TILES[precision]:
            rec = lpx.record(precision, gemm=tiles)
            print(f"case: gemm {M}x{N}x{K} {lpx.describe(rec)}", flush=True)
            C = lpx.gemm(Ad, Bd, record=rec)
            torch.cuda.synchronize()
            check(C.double().cpu().numpy(), A, B, precision)


def test_gemm_integer_exact_and_identity():
    A, B = inputs.integer_gemm_inputs(150, 90, 70, seed=2)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    Ad, Bd = to_dev(A), to_dev(B)
    for precision, tl in TILES.items():
        for tiles in tl[:3]:
            C = lpx.gemm(Ad, Bd, record=lpx.record(precision, gemm=tiles))
            torch.cuda.synchronize()
            assert np.array_equal(C.double().cpu().numpy(), exact), (precision, tiles)
    I = torch.eye(70, device="cuda")
    C = lpx.gemm(I, Bd, record=None)
    torch.cuda.synchronize()
    assert torch.equal(C, Bd)


def test_gemm_strided_rows():
    A, B = inputs.gemm_inputs(70, 50, 40, seed=3)
    Ab = torch.zeros((70, 44), device="cuda")
    Ab[:, :40] = to_dev(A)
    Cb = torch.full((70, 53), 7.0, device="cuda")
    lpx.gemm(Ab[:, :40], to_dev(B), C=Cb[:, :50], record=lpx.record("fp32", gemm=(64, 64, 32)))
    torch.cuda.synchronize()
    check(Cb[:, :50].double().cpu().numpy(), A, B, "fp32")
    assert bool((Cb[:, 50:] == 7.0).all())


@pytest.mark.parametrize("shape", [(4096, 4096, 4096), (8192, 1024, 4096)])
def test_gemm_full_size_every_tile(shape):
    """Full-size shapes, where the work-groups' XCD-grouped tile order runs
    (its remap applies only when the tile count is a multiple of 8): C is
    filled with NaN and none may remain; one row of every 128-row m-tile and
    a 4-column stripe (all rows) of every 128-column n-tile are checked
    against the FP64 oracle and its emulation of the precision."""
    M, N, K = shape
    A, B = inputs.gemm_inputs(M, N, K, seed=0)
    Ad, Bd = to_dev(A), to_dev(B)
    rows = [t * 128 + (37 * t + 5) % 128 for t in range(M // 128)]
    cols = [t * 128 + c for t in range(N // 128) for c in ((29 * t + 3) % 125,)]
    cols = sorted(c + d for c in cols for d in range(4))
    # row m of C depends only on row m of A, column n only on column n of B
    Ar = np.ascontiguousarray(A[rows])
    Bc = np.ascontiguousarray(B[:, cols])
    refs = {prec: (oracle.gemm(Ar, B, prec), oracle.gemm(A, Bc, prec))
            for prec in ("fp32", "bf16", "bf16x3")}
    cases = [("fp32", (128, 128, 64)), ("fp32", (128, 128, 32)), ("bf16", (128, 128, 32)),
             ("bf16x3", (128, 128, 32))]
    cases += [(prec, t) for prec, tl in PRESPLIT.items() for t in tl]
    for precision, tiles in cases:
        rec = lpx.record(precision, gemm=tiles)
        print(f"case: gemm full {shape} {lpx.describe(rec)}", flush=True)
        C = torch.full((M, N), float("nan"), device="cuda")
        lpx.gemm(Ad, Bd, C=C, record=rec)
        torch.cuda.synchronize()
        assert not bool(torch.isnan(C).any()), ("unwritten tiles", lpx.describe(rec))
        got_r = C[rows].double().cpu().numpy()
        got_c = C[:, cols].double().cpu().numpy()
        for got, ref, emu in ((got_r, refs["fp32"][0], refs[precision][0]),
                              (got_c, refs["fp32"][1], refs[precision][1])):
            err = oracle.rel_err(got, ref)
            assert err <= TOL[precision], (precision, tiles, err)
            if precision != "fp32":
                assert oracle.rel_err(got, emu) <= emu_tol(K), (precision, tiles)
        del C


@pytest.mark.parametrize("precision", ("bf16", "bf16x3"))
def test_gemm_presplit_strided_and_default(precision):
    """The pre-split path (the reduced precisions' default tiling, and the
    256-row tilings) with row strides that are not multiples of 4 and a
    ragged K, and the untouched columns of C past N."""
    A, B = inputs.gemm_inputs(300, 270, 45, seed=4)
    Ab = torch.zeros((300, 47), device="cuda")
    Ab[:, :45] = to_dev(A)
    Bb = torch.zeros((45, 273), device="cuda")
    Bb[:, :270] = to_dev(B)
    for tiles in [(0, 0, 0)] + PRESPLIT[precision]:
        rec = lpx.record(precision, gemm=tiles)
        print(f"case: gemm strided 300x270x45 {lpx.describe(rec)}", flush=True)
        Cb = torch.full((300, 275), 7.0, device="cuda")
        lpx.gemm(Ab[:, :45], Bb[:, :270], C=Cb[:, :270], record=rec)
        torch.cuda.synchronize()
        check(Cb[:, :270].double().cpu().numpy(), A, B, precision)
        assert bool((Cb[:, 270:] == 7.0).all())


@pytest.mark.parametrize("precision", ("bf16", "bf16x3"))
def test_gemm_presplit_k_zero(precision):
    """K = 0 with a pre-split tiling: nothing to split, C is all zeros (the
    general kernel writes them)."""
    A = torch.empty((300, 0), device="cuda")
    B = torch.empty((0, 270), device="cuda")
    for tiles in PRESPLIT[precision]:
        C = torch.full((300, 270), 7.0, device="cuda")
        lpx.gemm(A, B, C=C, record=lpx.record(precision, gemm=tiles))
        torch.cuda.synchronize()
        assert bool((C == 0).all()), tiles
