"""lpx_contract_noalloc, the entry point for callers that cannot allocate,
against lpx_contract through the C ABI on the GPU.

Both run the same kernels, so the outputs must agree bit for bit; the
outputs are written over a NaN sentinel, so a tile left unwritten fails the
comparison.  Each record runs twice in a row, the second call on a smaller
problem, so the second call reads the scratch array the first one left
behind.  One case is also checked against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from paper_1405_7470_amd import inputs, lpx
from tests.gpu_util import as_em, check_against_oracle, to_dev

pytestmark = pytest.mark.gpu

# (precision, tile_e, prefetch, unroll): D from its arrangement in scratch
# (prefetch 0, 2, 10), D in LDS (1, 3, 11) and D in registers (14, 6)
RECORDS = [("fp32", 16, 0, 1), ("fp32", 32, 2, 2), ("fp32", 64, 10, 1), ("bf16x3", 16, 0, 1),
           ("bf16x3", 64, 10, 2), ("bf16", 32, 0, 4), ("fp32", 64, 14, 1), ("fp32", 32, 3, 1),
           ("bf16x3", 64, 6, 1)]
# the second problem of each pair is smaller than the first
SHAPES = [((3, 56, 50_003), (3, 20, 1_001)), ((3, 120, 9_000), (3, 35, 777))]


def _pair(K, Np, E, layout, rec, seed):
    D, u = inputs.contraction_inputs(K, Np, E, seed=seed, layout=layout)
    Dd, ud = to_dev(D), to_dev(u)
    shape = lpx.out_shape(K, Np, E, layout)
    ref = torch.full(shape, float("nan"), device="cuda")
    lpx.contract(Dd, ud, out=ref, layout=layout, record=rec)
    out = torch.full(shape, float("nan"), device="cuda")
    lpx.contract_noalloc(Dd, ud, out, layout=layout, record=rec)
    torch.cuda.synchronize()
    return D, u, ref, out


@pytest.mark.parametrize("layout", ["em", "dm"])
@pytest.mark.parametrize("prec,tile,pf,un", RECORDS)
def test_noalloc_matches_contract_twice(layout, prec, tile, pf, un):
    rec = lpx.record(prec, tile, pf, un)
    for pair in SHAPES:
        for call, (K, Np, E) in enumerate(pair):
            if lpx.contract_validate(lpx.ContractDesc(K, Np, E, lpx.LAYOUT[layout], 0, 1 << 32,
                                                      1 << 40, 1 << 44), rec) != lpx.OK:
                continue  # a record this shape cannot run (LDS or register limits)
            print(f"noalloc {layout} {lpx.describe(rec)} K={K} Np={Np} E={E} call {call}",
                  flush=True)
            D, u, ref, out = _pair(K, Np, E, layout, rec, seed=call)
            assert not torch.isnan(ref).any()
            assert torch.equal(out, ref), (layout, lpx.describe(rec), K, Np, E)


def test_noalloc_against_oracle():
    rec = lpx.default_record("fp32")
    for K, Np, E in ((3, 56, 4_099), (3, 10, 333)):
        D, u, ref, out = _pair(K, Np, E, "em", rec, seed=7)
        check_against_oracle(D, u, as_em(out, "em"), "em", "fp32")
        assert torch.equal(out, ref)
