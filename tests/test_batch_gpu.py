"""Ragged batch as one graph of persistent launches (one per kernel the
records select): bit-identical to separate lpx_contract calls with the same
records, within tolerance of the oracle, replayable with new buffers; mixed
precisions and layouts, runs that split a large instance over many
work-groups, instances smaller than a tile, records rejected like
lpx_contract rejects them; plus sampled instances of the 512-instance
workload."""
import numpy as np
import pytest
import torch

from paper_1405_7470_amd import inputs, lpx
from tests.gpu_util import as_em, check_against_oracle, to_dev

pytestmark = pytest.mark.gpu


def make_items(shapes, seed, layout="em", K=3):
    host = inputs.ragged_batch_inputs(shapes, K=K, seed=seed)
    items = []
    for D, u in host:
        uu = u if layout == "em" else np.ascontiguousarray(u.T)
        Dd, ud = to_dev(D), to_dev(uu)
        out = torch.empty(lpx.out_shape(K, D.shape[1], u.shape[0], layout), device="cuda")
        items.append((Dd, ud, out, layout))
    return host, items


def valid_records(items, rng, precisions, prefetches=(0, 1, 2, 3, 4, 6, 10, 11, 14)):
    """A random record per item; where its storage does not fit the
    instance, the same record with prefetch 0 (always valid)."""
    recs = []
    for (D, u, out, lay) in items:
        K, Np = D.shape[0], D.shape[1]
        E = u.shape[0] if lay == "em" else u.shape[1]
        rec = lpx.record(str(rng.choice(precisions)), int(rng.choice([16, 32, 64])),
                         int(rng.choice(prefetches)), int(rng.choice([1, 2, 4])))
        if lpx.lds_bytes(K, Np, E, lay, rec)[0] != lpx.OK:
            rec = lpx.record(lpx.describe(rec).split()[0], rec.tile_e, 0, rec.unroll)
        recs.append(rec)
    return recs


def check_batch(items, recs, host, precisions):
    for (D, u, out, lay), rec, (Dh, uh) in zip(items, recs, host):
        ref = lpx.contract(D, u, layout=lay, record=rec)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), lpx.describe(rec)
        uu = uh if lay == "em" else np.ascontiguousarray(uh.T)
        check_against_oracle(Dh, uu, as_em(out, lay), lay, precisions[lpx.describe(rec).split()[0]])


@pytest.mark.parametrize("precision", ("fp32", "bf16x3", "bf16"))
@pytest.mark.parametrize("layout", ("em", "dm"))
def test_batch_bitwise_equals_separate_calls(precision, layout):
    shapes = inputs.ragged_shapes(n=40, seed=7, lo=1, hi=3000)
    host, items = make_items(shapes, seed=3, layout=layout)
    recs = valid_records(items, np.random.default_rng(1), [precision])
    print(f"case: batch {precision} {layout} n={len(shapes)}", flush=True)
    b = lpx.Batch(items, recs)
    torch.cuda.synchronize()
    assert b.info()["tiles"] == sum(
        (E + r.tile_e - 1) // r.tile_e for (_, E), r in zip(shapes, recs))
    check_batch(items, recs, host, {precision: precision})
    b.destroy()


def test_batch_mixed_precisions_layouts_and_records():
    """One batch whose instances differ in precision, layout and record:
    every instance runs its own record's kernel."""
    shapes = inputs.ragged_shapes(n=36, seed=21, lo=1, hi=5000)
    host_e, items_e = make_items(shapes[:18], seed=8, layout="em")
    host_d, items_d = make_items(shapes[18:], seed=9, layout="dm")
    host, items = host_e + host_d, items_e + items_d
    precs = ["fp32", "bf16", "bf16x3"]
    recs = valid_records(items, np.random.default_rng(5), precs)
    print(f"case: batch mixed n={len(items)}", flush=True)
    b = lpx.Batch(items, recs)
    torch.cuda.synchronize()
    assert b.info()["kernels"] > 3
    check_batch(items, recs, host, {p: p for p in precs})
    b.destroy()


def test_batch_runs_split_large_and_tiny_instances():
    """A large instance cut into many runs over the work-groups, beside
    instances smaller than one tile."""
    shapes = [(56, 300000), (20, 5), (120, 3), (35, 70001), (84, 17)]
    host, items = make_items(shapes, seed=12)
    for rec in (lpx.record("fp32", 64, 14, 1), lpx.record("fp32", 32, 10, 2),
                lpx.record("bf16x3", 64, 6, 1), lpx.record("fp32", 16, 0, 4)):
        recs = valid_records(items, np.random.default_rng(0), ["fp32"], prefetches=(0,))
        recs[0] = rec  # the large instance (Np = 56) takes the record under test
        print(f"case: batch runs {lpx.describe(rec)}", flush=True)
        for (_, _, out, _) in items:
            out.fill_(float("nan"))
        b = lpx.Batch(items, recs)
        torch.cuda.synchronize()
        check_batch(items, recs, host, {"fp32": "fp32", "bf16x3": "bf16x3"})
        b.destroy()


def test_batch_replay_with_new_buffers_and_sentinel():
    shapes = inputs.ragged_shapes(n=25, seed=11, lo=10, hi=2000)
    host, items = make_items(shapes, seed=5)
    recs = [lpx.record("fp32", 32, 10, 1)] * len(shapes)
    b = lpx.Batch(items, recs)
    torch.cuda.synchronize()
    info = b.info()
    # one record: one kernel per i-block bound present (Np up to 32, 64, 128)
    assert info["kernels"] == len({2 if Np <= 32 else 4 if Np <= 64 else 8 for Np, _ in shapes})
    assert info["tiles"] == sum((E + 31) // 32 for _, E in shapes)
    # new inputs and NaN-filled outputs, same shapes: replay the graph
    host2, items2 = make_items(shapes, seed=6)
    for (_, _, out, _) in items2:
        out.fill_(float("nan"))
    for _ in range(3):  # several replays, with eager work in between
        b.submit(items2)
        torch.cuda.synchronize()
        _ = torch.ones(10, device="cuda").sum().item()
        for (D, u, out, lay), (Dh, uh) in zip(items2, host2):
            assert not torch.isnan(out).any()
            check_against_oracle(Dh, uh, as_em(out, lay), lay, "fp32")
    # a replay without descriptors reuses the last table (items2)
    ref = [out.clone() for (_, _, out, _) in items2]
    for (_, _, out, _) in items2:
        out.fill_(float("nan"))
    b.submit()
    torch.cuda.synchronize()
    for (_, _, out, _), r in zip(items2, ref):
        assert torch.equal(out, r)
    b.destroy()


def test_batch_rejects_unfit_records_and_changed_shapes():
    # D of K = 6, Np = 120 (345,600 bytes) cannot be staged in LDS: rejected,
    # as lpx_contract rejects it
    _, items6 = make_items([(120, 100), (20, 50)], seed=1, K=6)
    with pytest.raises(lpx.LpxError) as ei:
        lpx.Batch(items6, [lpx.record("fp32", 16, 1, 1), lpx.record("fp32")])
    assert ei.value.status == lpx.ERR_UNSUPPORTED
    assert "instance 0" in str(ei.value)
    shapes = [(20, 100), (56, 50)]
    _, items = make_items(shapes, seed=1)
    b = lpx.Batch(items, None)
    _, items_bad = make_items([(20, 100), (56, 51)], seed=1)
    with pytest.raises(lpx.LpxError) as ei:
        b.submit(items_bad)
    assert ei.value.status == lpx.ERR_INVALID_ARG
    b.destroy()


def test_batch_512_instances_sampled():
    """The 512-instance workload (Np over {10,...,120}, E log-uniform in
    [1024, 65536], seed 0): a sample of instances checked bit-for-bit
    against lpx_contract and against the oracle."""
    shapes = inputs.ragged_shapes(n=512, seed=0)
    host, items = make_items(shapes, seed=0)
    b = lpx.Batch(items, None)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for i in sorted(set(int(x) for x in rng.integers(0, 512, 12)) | {0, 511}):
        D, u, out, lay = items[i]
        ref = lpx.contract(D, u, layout=lay)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), i
        Dh, uh = host[i]
        n = min(64, uh.shape[0])
        check_against_oracle(Dh, uh, as_em(out[:, :n, :], "em"), "em", "fp32", e0=0)
    b.destroy()


def test_batch_six_operators():
    """K = 6 (stacked rows up to 720 at Np = 120): every record that fits
    each instance, bit-identical to separate calls."""
    shapes = [(120, 700), (56, 333), (10, 1500), (84, 65)]
    host, items = make_items(shapes, seed=9, K=6)
    recs = valid_records(items, np.random.default_rng(3), ["fp32"])
    b = lpx.Batch(items, recs)
    torch.cuda.synchronize()
    check_batch(items, recs, host, {"fp32": "fp32"})
    b.destroy()


def test_batch_tune_groups_and_bitwise():
    """lpx_batch_tune: one record per (K, Np, layout) group, each valid for
    all of its instances; the batch built with them matches separate calls."""
    shapes = [(20, 900), (20, 3000), (56, 1200), (56, 40), (120, 700), (120, 2500)]
    host, items = make_items(shapes, seed=4)
    recs = lpx.batch_tune(items, "fp32", warmup=1, reps=3)
    assert len(recs) == len(items)
    for a, b in ((0, 1), (2, 3), (4, 5)):
        assert lpx.describe(recs[a]) == lpx.describe(recs[b])
    # the batch ignores the tile order: only cyclic-order records are timed
    assert all(r.order == 0 for r in recs)
    b = lpx.Batch(items, recs)
    torch.cuda.synchronize()
    check_batch(items, recs, host, {"fp32": "fp32"})
    b.destroy()
