"""Parity of every contraction variant (HIP path, through the C ABI) with
the FP64 oracle, at sizes the oracle finishes in seconds, plus coverage,
determinism and exactness checks."""
import numpy as np
import pytest
import torch

import oracle
from paper_1405_7470_amd import inputs, lpx
from tests.gpu_util import as_em, check_against_oracle, dev, to_dev

pytestmark = pytest.mark.gpu

PRECS = ("fp32", "bf16x3", "bf16")
LAYOUTS = ("em", "dm")


def supported(K, Np, E, layout, rec):
    """Records that validation accepts for the shape (some storage choices,
    e.g. D in registers, only exist for part of the shapes)."""
    st, _ = lpx.lds_bytes(K, Np, E, layout, rec)
    return st == lpx.OK


def run(D, u, layout, rec):
    Dd, ud = to_dev(D), to_dev(u)
    out = lpx.contract(Dd, ud, layout=layout, record=rec)
    torch.cuda.synchronize()
    return out


def test_untuned_plain_fp32_small_config():
    """K=3 operators of 20x20, E=4096, seed 0, element-major, untuned."""
    D, u = inputs.contraction_inputs(3, 20, 4096, seed=0)
    print("case: untuned fp32 K=3 Np=20 E=4096", flush=True)
    out = run(D, u, "em", None)
    err = check_against_oracle(D, u, as_em(out, "em"), "em", "fp32")
    print(f"rel_err={err:.3e}")


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("layout", LAYOUTS)
def test_every_record_matches_oracle(precision, layout):
    """All 18 records; Np spans 1..3 and 4 i-blocks, E has a ragged tail."""
    for Np, E in ((20, 1000), (56, 333), (35, 77)):
        D, u = inputs.contraction_inputs(3, Np, E, seed=Np, layout=layout)
        for rec in lpx.enumerate_records(3, Np, E, layout, precision):
            if not supported(3, Np, E, layout, rec):
                continue
            print(f"case: {precision} {layout} Np={Np} E={E} {lpx.describe(rec)}", flush=True)
            out = run(D, u, layout, rec)
            check_against_oracle(D, u, as_em(out, layout), layout, precision)


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("layout", LAYOUTS)
def test_edge_shapes(precision, layout):
    """Np across the i-block classes, E below/at/above tile multiples."""
    shapes = [(1, 1), (1, 17), (10, 15), (16, 16), (17, 65), (64, 64), (84, 129),
              (120, 31), (128, 70)]
    recs = [lpx.record(precision, t, p, un) for (t, p, un) in
            ((16, 0, 1), (64, 0, 4), (32, 1, 2), (64, 3, 1), (16, 2, 4), (32, 4, 1),
             (32, 6, 1), (32, 10, 2), (64, 11, 1), (16, 14, 1))]
    for Np, E in shapes:
        D, u = inputs.contraction_inputs(2, Np, E, seed=E, layout=layout)
        for rec in recs:
            if not supported(2, Np, E, layout, rec):
                continue
            print(f"case: edge {precision} {layout} Np={Np} E={E} {lpx.describe(rec)}", flush=True)
            out = run(D, u, layout, rec)
            check_against_oracle(D, u, as_em(out, layout), layout, precision)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_row_blocks_across_operators(layout):
    """The K operators are stacked into K*Np rows cut in blocks of 16: blocks
    that start in one operator and end in the next (Np not a multiple of 4
    or 16), a partial last block, and K up to 7."""
    recs = ((16, 0, 1), (32, 1, 1), (64, 3, 2), (32, 4, 1), (32, 6, 1), (32, 10, 1),
            (64, 11, 1), (32, 14, 1))
    E = 203
    for K, Np in ((1, 5), (3, 5), (5, 6), (7, 10), (3, 13), (4, 20), (5, 36), (3, 56),
                  (2, 120)):
        D, u = inputs.contraction_inputs(K, Np, E, seed=K * 1000 + Np, layout=layout)
        for precision in PRECS:
            for t, p, un in recs:
                rec = lpx.record(precision, t, p, un)
                if not supported(K, Np, E, layout, rec):
                    continue
                print(f"case: row blocks {precision} {layout} K={K} Np={Np} {lpx.describe(rec)}",
                      flush=True)
                out = run(D, u, layout, rec)
                check_against_oracle(D, u, as_em(out, layout), layout, precision)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_arranged_d_matches_lds_staged_d(layout):
    """Records that read D from memory read its MFMA-order arrangement
    written by a pre-pass; the same fragments staged in LDS (prefetch bit 0)
    must give identical bits, at shapes where both exist (FP32 and bf16x3
    Np = 84, bf16 Np = 120), with ragged tiles."""
    for precision, Np in (("fp32", 84), ("bf16", 120), ("bf16x3", 84)):
        D, u = inputs.contraction_inputs(3, Np, 777, seed=Np, layout=layout)
        ref_rec = lpx.record(precision, 16, 1, 1)
        assert supported(3, Np, 777, layout, ref_rec)
        ref = run(D, u, layout, ref_rec)
        check_against_oracle(D, u, as_em(ref, layout), layout, precision)
        for t, p, un in ((16, 0, 1), (64, 0, 4), (32, 2, 2), (64, 10, 1)):
            rec = lpx.record(precision, t, p, un)
            if not supported(3, Np, 777, layout, rec):
                continue
            print(f"case: arranged D {precision} {layout} Np={Np} {lpx.describe(rec)}", flush=True)
            assert torch.equal(run(D, u, layout, rec), ref), lpx.describe(rec)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_many_tiles_per_work_group(layout):
    """E large enough that every work-group walks several tiles (the
    staged pipelines' steady state and drain) with a ragged last tile.  All
    records of a precision sum in the same order, so every record must match
    the untuned default bit for bit; the default is checked against the
    oracle on sampled elements."""
    E = 200_003
    rng = np.random.default_rng(1)
    for Np in (20, 56, 84):
        D, u = inputs.contraction_inputs(3, Np, E, seed=Np, layout=layout)
        Dd, ud = to_dev(D), to_dev(u)
        for precision in PRECS:
            ref = lpx.contract(Dd, ud, layout=layout, record=lpx.default_record(precision))
            torch.cuda.synchronize()
            for s0 in [0, E - 51] + [int(x) for x in rng.integers(0, E - 51, 3)]:
                chunk = ref[:, s0:s0 + 51, :] if layout == "em" else ref[:, :, s0:s0 + 51]
                check_against_oracle(D, u, as_em(chunk, layout), layout, precision, e0=s0)
            for rec in lpx.enumerate_records(3, Np, E, layout, precision):
                if not rec.prefetch & 2 or not supported(3, Np, E, layout, rec):
                    continue
                print(f"case: many-tiles {precision} {layout} Np={Np} {lpx.describe(rec)}",
                      flush=True)
                out = lpx.contract(Dd, ud, layout=layout, record=rec)
                assert torch.equal(out, ref), lpx.describe(rec)
                del out
            del ref


@pytest.mark.parametrize("layout", LAYOUTS)
def test_integer_inputs_bitwise_for_every_record(layout):
    """Small-integer operands make every partial sum exact in FP32 and every
    operand exact in bf16: all records and precisions give the exact result."""
    K, Np, E = 3, 40, 203
    D, u = inputs.integer_contraction_inputs(K, Np, E, seed=1, layout=layout)
    ue = u if layout == "em" else u.T
    exact = np.einsum("kij,ej->kei", D.astype(np.int64), ue.astype(np.int64)).astype(np.float64)
    for precision in PRECS:
        for rec in lpx.enumerate_records(K, Np, E, layout, precision):
            if not supported(K, Np, E, layout, rec):
                continue
            out = as_em(run(D, u, layout, rec), layout)
            assert np.array_equal(out, exact), (precision, lpx.describe(rec))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_coverage_sentinel_and_canary(layout):
    """Every output written exactly once, nothing past the end: the output is
    pre-filled with NaN and followed by a 4 KiB canary."""
    K, Np, E = 3, 35, 1001
    D, u = inputs.contraction_inputs(K, Np, E, seed=5, layout=layout)
    Dd, ud = to_dev(D), to_dev(u)
    n = K * E * Np
    canary = 1024
    for precision in PRECS:
        for rec in lpx.enumerate_records(K, Np, E, layout, precision):
            if not supported(K, Np, E, layout, rec):
                continue
            buf = torch.full((n + canary,), float("nan"), device=dev())
            buf[n:] = 12345.0
            out = buf[:n].view(lpx.out_shape(K, Np, E, layout))
            lpx.contract(Dd, ud, out=out, layout=layout, record=rec)
            torch.cuda.synchronize()
            assert not torch.isnan(buf[:n]).any(), lpx.describe(rec)
            assert bool((buf[n:] == 12345.0).all()), lpx.describe(rec)


def test_determinism():
    D, u = inputs.contraction_inputs(3, 56, 5000, seed=8)
    Dd, ud = to_dev(D), to_dev(u)
    for precision in PRECS:
        rec = lpx.record(precision, 64, 1, 2)
        outs = [lpx.contract(Dd, ud, record=rec) for _ in range(3)]
        torch.cuda.synchronize()
        assert all(torch.equal(outs[0], o) for o in outs[1:])


def test_identity_operator_gives_u():
    K, Np, E = 3, 56, 999
    _, u = inputs.contraction_inputs(K, Np, E, seed=9)
    D = np.stack([np.eye(Np, dtype=np.float32)] * K)
    for rec in (lpx.record("fp32", 64, 1, 4), lpx.default_record()):
        out = as_em(run(D, u, "em", rec), "em")
        for k in range(K):
            assert np.array_equal(out[k], u.astype(np.float64))


def test_layouts_agree():
    K, Np, E = 3, 56, 4099
    D, u = inputs.contraction_inputs(K, Np, E, seed=12)
    for precision in PRECS:
        rec = lpx.record(precision, 32, 1, 1)
        a = as_em(run(D, u, "em", rec), "em")
        b = as_em(run(D, np.ascontiguousarray(u.T), "dm", rec), "dm")
        assert oracle.rel_err(a, b) <= 1e-6


def test_non_default_stream():
    D, u = inputs.contraction_inputs(3, 20, 3000, seed=13)
    Dd, ud = to_dev(D), to_dev(u)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = lpx.contract(Dd, ud, record=lpx.record("fp32", 32, 1, 2))
    s.synchronize()
    check_against_oracle(D, u, as_em(out, "em"), "em", "fp32")


def test_split_bf16_bitwise():
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(100003) * np.exp2(rng.integers(-60, 60, 100003))).astype(np.float32)
    hi, lo = lpx.split_bf16(to_dev(x))
    torch.cuda.synchronize()
    ohi, olo = oracle.split_bf16(x)
    ghi = (hi.cpu().numpy().astype(np.int32) & 0xFFFF).astype(np.uint32) << 16
    glo = (lo.cpu().numpy().astype(np.int32) & 0xFFFF).astype(np.uint32) << 16
    assert np.array_equal(ghi, ohi.view(np.uint32))
    assert np.array_equal(glo, olo.view(np.uint32))


def test_errors_raise_and_alias_detected():
    D = torch.zeros((3, 20, 20), device=dev())
    u = torch.zeros((100, 20), device=dev())
    with pytest.raises(lpx.LpxError) as ei:
        lpx.contract(D, u, record=lpx.record("fp32", 64, 0, 1, assume_tile_divides=1))
    assert ei.value.status == lpx.ERR_ASSUMPTION
    buf = torch.zeros(3 * 100 * 20 + 100 * 20, device=dev())
    u2 = buf[:2000].view(100, 20)
    out = buf[1000:1000 + 6000].view(3, 100, 20)  # overlaps u2
    with pytest.raises(lpx.LpxError) as ei:
        lpx.contract(D, u2, out=out)
    assert ei.value.status == lpx.ERR_ALIAS


def test_autotune_picks_the_fastest_and_caches_it():
    K, Np, E = 3, 20, 20000
    D, u = inputs.contraction_inputs(K, Np, E, seed=14)
    Dd, ud = to_dev(D), to_dev(u)
    lpx.tune_cache_clear()
    best, times = lpx.autotune(Dd, ud, layout="em", precision="bf16x3", warmup=1, reps=3)
    recs = lpx.enumerate_records(K, Np, E, "em", "bf16x3")
    assert len(times) == len(recs)
    finite = [t for t in times if np.isfinite(t)]
    assert finite and min(finite) == times[recs.index(best)]
    # the tuner overwrote out with a valid result of the last candidate
    out = lpx.contract(Dd, ud, record=best)
    torch.cuda.synchronize()
    check_against_oracle(D, u, as_em(out, "em"), "em", "bf16x3")


def test_stream_probe():
    x = torch.arange(1 << 16, dtype=torch.float32, device=dev())
    for fanout in (1, 3):
        y = torch.empty(fanout * x.numel(), device=dev())
        lpx.stream_probe(x, y, fanout)
        torch.cuda.synchronize()
        assert torch.equal(y.view(fanout, -1), x.expand(fanout, -1))
