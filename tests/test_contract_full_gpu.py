"""Parity at the full scale (K=3, Np=56, E=2^20), both layouts, FP32 and
bf16x3, in the launch configuration the benchmark times: every output is
written over a NaN sentinel and none may remain (the persistent grid's tile
walk covers every element), and sampled element chunks (first, last and
random) are checked against the FP64 oracle."""
import numpy as np
import pytest
import torch

from paper_1405_7470_amd import inputs, lpx
from tests.gpu_util import check_against_oracle, to_dev

pytestmark = pytest.mark.gpu

K, NP, E = 3, 56, 1 << 20


@pytest.mark.parametrize("layout", ("em", "dm"))
def test_full_scale_sampled(layout):
    D, u = inputs.contraction_inputs(K, NP, E, seed=0, layout=layout)
    Dd, ud = to_dev(D), to_dev(u)
    rng = np.random.default_rng(0)
    starts = [0, E - 97] + [int(s) for s in rng.integers(0, E - 64, 6)]
    for precision in ("fp32", "bf16x3"):
        # the benchmark's picks (tile 64 and 32 with u, D and output staged or
        # held, and tile 64 with D in registers) and a spread of other records
        for rec in (lpx.default_record(precision), lpx.record(precision, 64, 14, 1),
                    lpx.record(precision, 32, 14, 1), lpx.record(precision, 64, 6, 1),
                    lpx.record(precision, 64, 14, 2), lpx.record(precision, 64, 1, 2),
                    lpx.record(precision, 32, 3, 4), lpx.record(precision, 16, 2, 1),
                    lpx.record(precision, 32, 6, 1), lpx.record(precision, 64, 4, 1),
                    lpx.record(precision, 64, 10, 4)):
            print(f"case: full {layout} {lpx.describe(rec)}", flush=True)
            out = torch.full(lpx.out_shape(K, NP, E, layout), float("nan"), device="cuda")
            lpx.contract(Dd, ud, out=out, layout=layout, record=rec)
            torch.cuda.synchronize()
            assert not bool(torch.isnan(out).any()), ("unwritten outputs", lpx.describe(rec))
            for s0 in starts:
                n = min(97, E - s0)
                if layout == "em":
                    chunk = out[:, s0:s0 + n, :].double().cpu().numpy()
                else:
                    chunk = out[:, :, s0:s0 + n].double().cpu().numpy().transpose(0, 2, 1)
                check_against_oracle(D, u, chunk, layout, precision, e0=s0)
            del out
