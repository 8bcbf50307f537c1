"""The dG volume term (lpx_dg_volume) against the FP64 oracle on the GPU.

out[d,e,i] = sum_k G(e,d,k) sum_j D[k][i][j] u[e][j]: every staged-output
record (the epilogue runs in the store waves) in every precision and layout
on ragged shapes, written over a NaN sentinel; the epilogue against the
plain contraction of the same record combined with G on the host; the
identity metric bit for bit against lpx_contract; small-integer inputs
exactly; and the full workload size on sampled elements.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1405_7470_amd import inputs, lpx
from tests.gpu_util import TOL, emu_tol, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(3, 56, 517), (3, 20, 333), (2, 35, 129), (1, 10, 77), (3, 16, 64), (3, 84, 150),
          (3, 120, 70)]


def _records(precision):
    for tile in (16, 32, 64):
        for pf, unrolls in ((10, (1, 2, 4)), (11, (1, 4)), (14, (1,))):
            for un in unrolls:
                yield lpx.record(precision, tile, pf, un)


def _fits(K, Np, E, layout, rec):
    d = lpx.DgDesc(K, Np, E, lpx.LAYOUT[layout], 0, 1 << 32, 1 << 40, 1 << 41, 1 << 44)
    return lpx.dg_volume_validate(d, rec)[0] == lpx.OK


def _as_em(out, layout):
    o = out.detach().cpu().numpy().astype(np.float64)
    return o if layout == "em" else np.ascontiguousarray(o.transpose(0, 2, 1))


def _run(D, u, G, layout, rec):
    K, Np = D.shape[0], D.shape[1]
    E = u.shape[0] if layout == "em" else u.shape[1]
    out = torch.full(lpx.out_shape(K, Np, E, layout), float("nan"), device="cuda")
    lpx.dg_volume(to_dev(D), to_dev(u), to_dev(G), out=out, layout=layout, record=rec)
    torch.cuda.synchronize()
    assert not bool(torch.isnan(out).any()), ("unwritten outputs", lpx.describe(rec))
    return out


def _check(y, D, u, G, layout, precision, e0=0):
    ne = y.shape[1]
    ref = oracle.dg_volume(D, u, G, layout, "fp32", e0, ne)
    err = oracle.rel_err(y, ref)
    assert err <= TOL[precision], (precision, err)
    if precision != "fp32":
        emu = oracle.dg_volume(D, u, G, layout, precision, e0, ne)
        # the metric mixes K sums: FP32 accumulation error grows by at most K
        assert oracle.rel_err(y, emu) <= 4 * emu_tol(D.shape[1]), precision
    return err


@pytest.mark.parametrize("layout", ["em", "dm"])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16"])
def test_dg_every_record(layout, precision):
    for K, Np, E in SHAPES:
        D, u, G = inputs.dg_volume_inputs(K, Np, E, seed=K * 1000 + Np, layout=layout)
        for rec in _records(precision):
            if not _fits(K, Np, E, layout, rec):
                continue
            print(f"case: dg {layout} {lpx.describe(rec)} K={K} Np={Np} E={E}", flush=True)
            out = _run(D, u, G, layout, rec)
            _check(_as_em(out, layout), D, u, G, layout, precision)


@pytest.mark.parametrize("layout", ["em", "dm"])
def test_dg_epilogue_against_contraction(layout):
    """The epilogue alone: lpx_dg_volume against lpx_contract of the same
    record (same reference derivatives, bit for bit) combined with G on the
    host in FP64; only the FP32 rounding of K products remains."""
    K, Np, E = 3, 56, 1000
    D, u, G = inputs.dg_volume_inputs(K, Np, E, seed=3, layout=layout)
    Gem = G if layout == "em" else np.ascontiguousarray(G.transpose(2, 0, 1))
    for rec in (lpx.record("fp32", 64, 14, 1), lpx.record("bf16x3", 32, 10, 2),
                lpx.record("fp32", 16, 11, 1)):
        out = _as_em(_run(D, u, G, layout, rec), layout)
        c = lpx.contract(to_dev(D), to_dev(u), layout=layout, record=rec)
        torch.cuda.synchronize()
        c = _as_em(c, layout)
        want = np.einsum("edk,kei->dei", Gem.astype(np.float64), c)
        bound = 4 * 2.0 ** -24 * np.einsum("edk,kei->dei", np.abs(Gem.astype(np.float64)),
                                          np.abs(c)) + 1e-30
        assert np.all(np.abs(out - want) <= bound), lpx.describe(rec)


@pytest.mark.parametrize("layout", ["em", "dm"])
def test_dg_identity_metric_is_the_contraction(layout):
    K, Np, E = 3, 35, 301
    D, u, _ = inputs.dg_volume_inputs(K, Np, E, seed=4, layout=layout)
    I = np.broadcast_to(np.eye(K, dtype=np.float32), (E, K, K)).copy()
    G = I if layout == "em" else np.ascontiguousarray(I.transpose(1, 2, 0))
    for rec in (lpx.record("fp32", 32, 10, 1), lpx.record("bf16x3", 64, 14, 1),
                lpx.record("bf16", 16, 11, 2)):
        out = _run(D, u, G, layout, rec)
        c = lpx.contract(to_dev(D), to_dev(u), layout=layout, record=rec)
        torch.cuda.synchronize()
        assert torch.equal(out, c), lpx.describe(rec)


def test_dg_integer_inputs_exact():
    K, Np, E = 3, 24, 95
    D, u = inputs.integer_contraction_inputs(K, Np, E, seed=5, bound=4)
    G = np.random.default_rng(6).integers(-3, 4, (E, K, K)).astype(np.float32)
    exact = np.einsum("edk,kij,ej->dei", G.astype(np.int64), D.astype(np.int64),
                      u.astype(np.int64)).astype(np.float64)
    for layout in ("em", "dm"):
        uu = u if layout == "em" else np.ascontiguousarray(u.T)
        GG = G if layout == "em" else np.ascontiguousarray(G.transpose(1, 2, 0))
        for precision in ("fp32", "bf16", "bf16x3"):
            for rec in (lpx.record(precision, 16, 10, 1), lpx.record(precision, 64, 14, 1)):
                out = _as_em(_run(D, uu, GG, layout, rec), layout)
                assert np.array_equal(out, exact), (layout, lpx.describe(rec))


@pytest.mark.parametrize("layout", ["em", "dm"])
def test_dg_full_size_sampled(layout):
    K, Np, E = 3, 56, 1 << 20
    D, u, G = inputs.dg_volume_inputs(K, Np, E, seed=0, layout=layout)
    rng = np.random.default_rng(1)
    starts = [0, E - 97] + [int(s) for s in rng.integers(0, E - 97, 4)]
    for rec in (lpx.record("fp32", 64, 14, 1), lpx.record("bf16x3", 64, 14, 1),
                lpx.record("fp32", 64, 10, 1), None):
        print(f"case: dg full {layout} {lpx.describe(rec) if rec else 'default'}", flush=True)
        out = _run(D, u, G, layout, rec)
        prec = lpx.PRECISION_NAME[rec.precision] if rec else "fp32"
        for s0 in starts:
            chunk = out[:, s0:s0 + 97, :] if layout == "em" else \
                out[:, :, s0:s0 + 97].transpose(1, 2)
            _check(chunk.double().cpu().numpy(), D, u, G, layout, prec, e0=s0)
        del out
