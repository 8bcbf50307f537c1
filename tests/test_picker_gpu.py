"""Learned picker end to end on the GPU at a small scale: exhaustive
timings -> training with the library's kernels -> model file -> learned
pick, checked against the FP64 oracle's pick on the same weights."""
import numpy as np
import pytest
import torch

from oracle import mlp
from paper_1405_7470_amd import lpx, picker

pytestmark = pytest.mark.gpu


def test_collect_train_pick(tmp_path):
    shapes = [{"K": 3, "Np": Np, "E": E, "layout": lay, "precision": prec}
              for Np, E, lay, prec in ((20, 3000, "em", "fp32"), (56, 5000, "dm", "bf16x3"),
                                       (35, 2048, "em", "bf16"), (84, 1500, "dm", "fp32"),
                                       (10, 4000, "em", "bf16x3"), (120, 1024, "em", "fp32"))]
    rows = picker.collect(shapes, flush_mb=64, reps=3, log=None)
    assert len(rows) >= 6 * 18
    assert all(r["us"] > 0 for r in rows)
    params, mean, std, hist = picker.train(rows, epochs=15, batch=64, log=None)
    assert np.all(np.isfinite(params)) and len(hist) >= 1
    path = tmp_path / "m.lpxpick"
    lpx.picker_save(path, params, mean, std)
    pk = lpx.Picker(path)
    for sh in shapes:
        rec = lpx.pick_variant(sh["K"], sh["Np"], sh["E"], sh["layout"], sh["precision"],
                               mode=lpx.PICK_LEARNED, picker=pk)
        cands = [r for r in lpx.enumerate_records(sh["K"], sh["Np"], sh["E"], sh["layout"],
                                                  sh["precision"])
                 if lpx.lds_bytes(sh["K"], sh["Np"], sh["E"], sh["layout"], r)[0] == lpx.OK]
        feats = np.array([lpx.features(sh["K"], sh["Np"], sh["E"], sh["layout"], r) for r in cands])
        p32, m32, s32 = pk.params()
        y, _ = mlp.forward(p32.astype(np.float64),
                           (feats - m32) / np.where(s32 == 0, 1, s32))
        # the GPU's pick is the oracle's argmin, or ties it to FP32 rounding
        i = cands.index(rec)
        assert y[i] <= y.min() + 1e-5 * max(1.0, abs(y.min())), (sh, lpx.describe(rec))
    pk.close()


def test_exhaustive_mode_uses_the_tuning_cache():
    D = torch.randn((3, 20, 20), device="cuda")
    u = torch.rand((3000, 20), device="cuda")
    lpx.tune_cache_clear()
    with pytest.raises(lpx.LpxError) as ei:
        lpx.pick_variant(3, 20, 3000, "em", "fp32", mode=lpx.PICK_EXHAUSTIVE)
    assert ei.value.status == lpx.ERR_NOT_TUNED
    best, _ = lpx.autotune(D, u, layout="em", precision="fp32", warmup=1, reps=3)
    rec = lpx.pick_variant(3, 20, 3000, "em", "fp32", mode=lpx.PICK_EXHAUSTIVE)
    assert rec == best
