"""Picker host logic on the CPU: model file round trip and rejection of
damaged files, the 13 features, and the pick modes that need no GPU."""
import ctypes
import math
import struct

import numpy as np
import pytest

from paper_1405_7470_amd import lpx


def write_model(path, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.1, lpx.MLP_PARAMS).astype(np.float32)
    m = rng.normal(0, 1, lpx.MLP_FEATURES).astype(np.float32)
    s = np.abs(rng.normal(1, 0.1, lpx.MLP_FEATURES)).astype(np.float32)
    lpx.picker_save(path, p, m, s)
    return p, m, s


def test_round_trip(tmp_path):
    f = tmp_path / "m.lpxpick"
    p, m, s = write_model(f)
    pk = lpx.Picker(f)
    p2, m2, s2 = pk.params()
    assert np.array_equal(p, p2) and np.array_equal(m, m2) and np.array_equal(s, s2)
    pk.close()
    assert f.stat().st_size == 8 + 16 + 4 * (2 * lpx.MLP_FEATURES + lpx.MLP_PARAMS) + 4


def damaged(tmp_path, how):
    f = tmp_path / "m.lpxpick"
    write_model(f)
    b = bytearray(f.read_bytes())
    if how == "truncated":
        b = b[:-10]
    elif how == "magic":
        b[0] ^= 0xFF
    elif how == "version":
        b[8:12] = struct.pack("<I", 2)
    elif how == "dims":
        b[16:20] = struct.pack("<I", 32)
    elif how == "checksum":
        b[200] ^= 0x01
    elif how == "nan":
        off = 24 + 4 * (24 + 7)
        b[off:off + 4] = struct.pack("<f", float("nan"))
        h = 2166136261
        for x in bytes(b[:-4]):
            h = ((h ^ x) * 16777619) & 0xFFFFFFFF
        b[-4:] = struct.pack("<I", h)
    f.write_bytes(bytes(b))
    return f


@pytest.mark.parametrize("how", ["truncated", "magic", "version", "dims", "checksum", "nan"])
def test_damaged_model_rejected(tmp_path, how):
    with pytest.raises(lpx.LpxError) as ei:
        lpx.Picker(damaged(tmp_path, how))
    assert ei.value.status == lpx.ERR_MODEL


def test_missing_model_rejected(tmp_path):
    with pytest.raises(lpx.LpxError) as ei:
        lpx.Picker(tmp_path / "nope")
    assert ei.value.status == lpx.ERR_MODEL


def test_features_by_hand():
    r = lpx.record("bf16x3", 32, 3, 4)
    f = lpx.features(3, 56, 1 << 20, "dm", r)
    # the 3 operators stacked are 168 rows: 11 row blocks of 16, 8 rows padding
    lds = 11 * 2 * 64 * 32 + 4 * (32 * 64 + 32) * 4
    expect = [math.log2(56), 20.0, 3.0, 1.0, 5.0, 1.0, 1.0, 2.0, 2.0, 8 / 176,
              3.0, lds / (160 * 1024), 0.0]
    assert np.allclose(f, expect, rtol=1e-6)
    f = lpx.features(3, 56, 1000, "em", lpx.record("fp32", 16, 6, 1))
    assert f[5] == 2.0 and f[6] == 1.0               # D in registers, u staged
    f = lpx.features(3, 56, 1000, "em", lpx.record("fp32", 16, 14, 1))
    assert f[5] == 2.0 and f[6] == 2.0               # ... and the output staged too
    f = lpx.features(3, 10, 1000, "em", lpx.default_record("fp32"))
    # Np = 10 rows are not 16-byte multiples, E = 1000 runs are
    assert f[9] == pytest.approx(2 / 32) and f[10] == 1.0
    assert f[5] == 0 and f[6] == 0 and f[11] == 0 and f[12] == 0
    r = lpx.default_record("fp32")
    r.order = 1
    assert lpx.features(3, 10, 1000, "em", r)[12] == 1.0  # blocked tile order


def test_pick_modes_without_gpu():
    r = lpx.pick_variant(3, 56, 1000, "em", "bf16", mode=lpx.PICK_UNTUNED, stream=0)
    assert (r.tile_e, r.prefetch, r.unroll, r.precision) == (16, 0, 1, 1)
    with pytest.raises(lpx.LpxError) as ei:
        lpx.pick_variant(3, 56, 1000, "em", "fp32", mode=lpx.PICK_LEARNED, picker=None, stream=0)
    assert ei.value.status == lpx.ERR_MODEL
    with pytest.raises(lpx.LpxError) as ei:
        lpx.pick_variant(3, 56, 1000, "em", "fp32", mode=7, stream=0)
    assert ei.value.status == lpx.ERR_INVALID_ARG


def test_widen_twelve_feature_model(tmp_path):
    """A 12-feature model file becomes a 13-feature one whose order weights
    are zero and whose other weights are unchanged (same predictions)."""
    from paper_1405_7470_amd import picker
    nh, nf = lpx.MLP_HIDDEN, 12
    n12 = nh * nf + nh + nh * nh + nh + nh + 1
    rng = np.random.default_rng(5)
    mean = rng.normal(0, 1, nf).astype("<f4")
    std = np.abs(rng.normal(1, 0.1, nf)).astype("<f4")
    p = rng.normal(0, 0.1, n12).astype("<f4")
    old = tmp_path / "m12"
    old.write_bytes(b"\0" * 24 + mean.tobytes() + std.tobytes() + p.tobytes() + b"\0" * 4)
    new = tmp_path / "m13"
    picker.widen_model(str(old), str(new))
    q, m, s = lpx.Picker(new).params()
    W1 = q[:nh * 13].reshape(nh, 13)
    assert np.array_equal(W1[:, :12], p[:nh * 12].reshape(nh, 12)) and not W1[:, 12].any()
    assert np.array_equal(q[nh * 13:], p[nh * 12:])
    assert np.array_equal(m, np.append(mean, 0)) and np.array_equal(s, np.append(std, 1))
    with pytest.raises(ValueError):
        picker.widen_model(str(new), str(tmp_path / "x"))
