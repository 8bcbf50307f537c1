"""The 3D Coulomb potential (lpx_coulomb) against the FP64 oracle on the GPU.

Every variant (source tile 256/512/1024, staged or not, 1/2/4 targets per
thread) in both storage layouts: within the componentwise bound of FP32
evaluation, bit-identical across variants (each target sums its pairs in
source order), edge sizes around the tiles, coincident points, and the
benchmark size on sampled targets.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1405_7470_amd import inputs, lpx
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _abs_charges(sources, layout):
    s = sources.copy()
    if layout == "em":
        s[:, 3] = np.abs(s[:, 3])
    else:
        s[3] = np.abs(s[3])
    return s


def check(phi, tg, sr, layout, t0=0):
    """|phi - ref| <= (ns + 16) 2^-24 sum_s |q_s| / r_ts: FP32 rounding of the
    differences, the squared distance, v_rsq_f32 and the running sum, each
    bounded by a few units of 2^-24 of the pair's |q| / r."""
    n = len(phi)
    ns = sr.shape[0] if layout == "em" else sr.shape[1]
    ref = oracle.coulomb(tg, sr, layout, t0, n)
    absref = oracle.coulomb(tg, _abs_charges(sr, layout), layout, t0, n)
    bound = (ns + 16) * 2.0 ** -24 * absref + 1e-30
    err = np.abs(phi.astype(np.float64) - ref)
    assert np.all(err <= bound), float(np.max(err / bound))
    return oracle.rel_err(phi, ref)


def _run(tg, sr, layout, rec):
    nt = tg.shape[0] if layout == "em" else tg.shape[1]
    phi = torch.full((nt,), float("nan"), device="cuda")
    lpx.coulomb(to_dev(tg), to_dev(sr), phi, layout=layout, record=rec)
    torch.cuda.synchronize()
    return phi.cpu().numpy()


@pytest.mark.parametrize("layout", ["em", "dm"])
def test_every_variant(layout):
    tg, sr = inputs.coulomb_inputs(3001, 1500, seed=1, layout=layout)
    first = None
    for rec in lpx.coulomb_records():
        print(f"case: coulomb {layout} {lpx.describe(rec)}", flush=True)
        phi = _run(tg, sr, layout, rec)
        assert not np.isnan(phi).any()
        err = check(phi, tg, sr, layout)
        assert err <= 1e-5, err
        if first is None:
            first = phi
        assert np.array_equal(phi, first), lpx.describe(rec)


@pytest.mark.parametrize("layout", ["em", "dm"])
def test_edge_sizes(layout):
    rec_list = [None, lpx.record("fp32", 64, 2, 4), lpx.record("fp32", 16, 2, 2),
                lpx.record("fp32", 32, 0, 4)]
    for nt, ns in ((1, 1), (1, 1023), (5, 1024), (257, 1025), (1025, 255), (4097, 2049)):
        tg, sr = inputs.coulomb_inputs(nt, ns, seed=nt + ns, layout=layout)
        for rec in rec_list:
            print(f"case: coulomb {layout} nt={nt} ns={ns} "
                  f"{lpx.describe(rec) if rec else 'default'}", flush=True)
            phi = _run(tg, sr, layout, rec)
            assert not np.isnan(phi).any()
            check(phi, tg, sr, layout)


def test_no_sources_and_coincident_points():
    tg, sr = inputs.coulomb_inputs(300, 0, seed=2)
    assert np.array_equal(_run(tg, sr, "em", None), np.zeros(300, np.float32))
    # targets at the source positions: each target's own pair contributes nothing
    _, sr = inputs.coulomb_inputs(1, 700, seed=3)
    tg = np.zeros((700, 4), np.float32)
    tg[:, :3] = sr[:, :3]
    for rec in (None, lpx.record("fp32", 64, 2, 4)):
        phi = _run(tg, sr, "em", rec)
        assert np.isfinite(phi).all()
        check(phi, tg, sr, "em")


def test_benchmark_size_sampled():
    nt, ns = 1 << 20, 1 << 15
    tg, sr = inputs.coulomb_inputs(nt, ns, seed=0, layout="em")
    rng = np.random.default_rng(0)
    starts = [0, nt - 64] + [int(s) for s in rng.integers(0, nt - 64, 4)]
    for rec in (lpx.record("fp32", 64, 2, 4), lpx.record("fp32", 16, 0, 1)):
        print(f"case: coulomb full {lpx.describe(rec)}", flush=True)
        phi = _run(tg, sr, "em", rec)
        assert not np.isnan(phi).any()
        for s0 in starts:
            check(phi[s0:s0 + 64], tg, sr, "em", t0=s0)
