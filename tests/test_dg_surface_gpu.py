"""The dG surface (lift) term (lpx_dg_surface) against the FP64 oracle.

Every precision, layout and lift variant (1, 2 or 4 element blocks per
wave) on tetrahedral face counts (4 faces of (N+1)(N+2)/2 nodes lifted to
(N+1)(N+2)(N+3)/6 nodes) and ragged element counts, over a NaN sentinel;
variants of one precision bit-identical; integer inputs exact; the
benchmark size on sampled elements.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1405_7470_amd import inputs, lpx
from tests.gpu_util import TOL, emu_tol, to_dev

pytestmark = pytest.mark.gpu

# (Np, nf, nfp): tetrahedra of degree 1, 3, 5, 7, a triangle-like case and
# a ragged one
SHAPES = [(4, 4, 3), (20, 4, 10), (56, 4, 21), (120, 4, 36), (10, 3, 4), (33, 5, 7)]


def _run(L, f, s, nf, layout, rec):
    Np = L.shape[0]
    E = f.shape[0] if layout == "em" else f.shape[1]
    out = torch.full((E, Np) if layout == "em" else (Np, E), float("nan"), device="cuda")
    lpx.dg_surface(to_dev(L), to_dev(f), to_dev(s), nf, out=out, layout=layout, record=rec)
    torch.cuda.synchronize()
    assert not bool(torch.isnan(out).any()), "unwritten outputs"
    o = out.cpu().numpy().astype(np.float64)
    return o if layout == "em" else np.ascontiguousarray(o.T)


def _check(y, L, f, s, nf, layout, precision, e0=0):
    ref = oracle.dg_surface(L, f, s, nf, layout, "fp32", e0, y.shape[0])
    err = oracle.rel_err(y, ref)
    assert err <= TOL[precision], (precision, err)
    if precision != "fp32":
        emu = oracle.dg_surface(L, f, s, nf, layout, precision, e0, y.shape[0])
        assert oracle.rel_err(y, emu) <= emu_tol(L.shape[1]), precision
    return err


@pytest.mark.parametrize("layout", ["em", "dm"])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16"])
def test_every_variant(layout, precision):
    for Np, nf, nfp in SHAPES:
        for E in (1, 77, 333):
            L, f, s = inputs.dg_surface_inputs(Np, nf, nfp, E, seed=Np + E, layout=layout)
            first = None
            for rec in lpx.surface_records(precision):
                print(f"case: lift {layout} {lpx.describe(rec)} Np={Np} nf={nf} nfp={nfp} E={E}",
                      flush=True)
                y = _run(L, f, s, nf, layout, rec)
                _check(y, L, f, s, nf, layout, precision)
                if first is None:
                    first = y
                assert np.array_equal(y, first), lpx.describe(rec)


def test_integer_inputs_exact():
    Np, nf, nfp, E = 24, 4, 6, 130
    rng = np.random.default_rng(3)
    L = rng.integers(-4, 5, (Np, nf * nfp)).astype(np.float32)
    f = rng.integers(-4, 5, (E, nf * nfp)).astype(np.float32)
    s = (2.0 ** rng.integers(-2, 3, (E, nf))).astype(np.float32)
    exact = (np.repeat(s, nfp, axis=1).astype(np.float64) * f) @ L.T.astype(np.float64)
    for precision in ("fp32", "bf16", "bf16x3"):
        for layout in ("em", "dm"):
            ff = f if layout == "em" else np.ascontiguousarray(f.T)
            ss = s if layout == "em" else np.ascontiguousarray(s.T)
            for rec in lpx.surface_records(precision):
                assert np.array_equal(_run(L, ff, ss, nf, layout, rec), exact)


@pytest.mark.parametrize("layout", ["em", "dm"])
def test_benchmark_size_sampled(layout):
    Np, nf, nfp, E = 56, 4, 21, 1 << 20
    L, f, s = inputs.dg_surface_inputs(Np, nf, nfp, E, seed=0, layout=layout)
    rng = np.random.default_rng(2)
    starts = [0, E - 97] + [int(x) for x in rng.integers(0, E - 97, 4)]
    for rec in (lpx.record("fp32", 64, 1, 1), lpx.record("bf16x3", 32, 1, 1)):
        print(f"case: lift full {layout} {lpx.describe(rec)}", flush=True)
        y = _run(L, f, s, nf, layout, rec)
        prec = lpx.PRECISION_NAME[rec.precision]
        for s0 in starts:
            _check(y[s0:s0 + 97], L, f, s, nf, layout, prec, e0=s0)
