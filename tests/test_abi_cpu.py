"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects every malformed call before any HIP call.

Calls that could launch work are only made with NULL pointers or zero
sizes; descriptors with stand-in addresses go to lpx_contract_validate,
which never launches or dereferences.
"""
import ctypes
import os
import re

import pytest

from paper_1405_7470_amd import lpx

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "lpx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lpx_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "lpx_contract" in names and "lpx_split_bf16" in names
    L = lpx.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_status_strings():
    assert "gfx950" in lpx.version()
    L = lpx.lib()
    assert L.lpx_status_string(0) == b"LPX_OK"
    assert L.lpx_status_string(lpx.ERR_ALIAS) == b"LPX_ERR_ALIAS"
    assert L.lpx_status_string(99) == b"LPX_ERR_UNKNOWN"


def test_default_record_is_the_untuned_variant():
    for prec in ("fp32", "bf16", "bf16x3"):
        r = lpx.default_record(prec)
        assert (r.version, r.tile_e, r.prefetch, r.unroll) == (1, 16, 0, 1)
        assert lpx.PRECISION_NAME[r.precision] == prec
        assert lpx.validate_record(r) == lpx.OK
    bad = lpx.Record()
    assert lpx.lib().lpx_record_default(7, ctypes.byref(bad)) == lpx.ERR_INVALID_ARG


def test_enumeration_canonical_order_and_truncation():
    recs = lpx.enumerate_records(3, 56, 1 << 20, "em", "bf16x3")
    assert len(recs) == 162 == lpx.MAX_RECORDS
    keys = [(r.order, r.tile_e, r.prefetch, r.unroll) for r in recs]
    assert keys == [(o, t, p, u) for o in (0, 1) for t in (16, 32, 64)
                    for p in (0, 1, 2, 3, 4, 6, 10, 11, 14) for u in (1, 2, 4)]
    assert all(lpx.PRECISION_NAME[r.precision] == "bf16x3" for r in recs)
    p = lpx.problem(3, 56, 1 << 20, "em", "fp32")
    arr = (lpx.Record * 4)()
    n = ctypes.c_int32()
    assert lpx.lib().lpx_record_enumerate(ctypes.byref(p), arr, 4, ctypes.byref(n)) == 0
    assert n.value == 162 and arr[3].unroll == 1 and arr[3].prefetch == 1


def test_describe():
    r = lpx.record("bf16", 64, 1, 4)
    assert lpx.describe(r) == "bf16 tile_e=64 prefetch=1 unroll=4 gemm=0x0x0"
    r = lpx.record("fp32", 32, 14, 1, order=1)
    assert lpx.describe(r) == "fp32 tile_e=32 prefetch=14 unroll=1 order=blocked gemm=0x0x0"


@pytest.mark.parametrize("field,value", [
    ("version", 2), ("precision", 3), ("tile_e", 8), ("tile_e", 128), ("prefetch", 5),
    ("prefetch", 7), ("prefetch", 8), ("prefetch", 9), ("prefetch", 12), ("prefetch", 15),
    ("unroll", 3), ("assume_tile_divides", 2), ("order", 2), ("reserved1", 1)])
def test_malformed_records_rejected(field, value):
    r = lpx.default_record()
    setattr(r, field, value)
    assert lpx.validate_record(r) == lpx.ERR_INVALID_ARG
    assert lpx.last_error()


A = 1 << 32  # stand-in, 16-byte aligned addresses (never dereferenced)


def desc(K=3, Np=56, E=1000, layout=0, D=A, u=A + (1 << 24), out=A + (1 << 28), reserved=0):
    return lpx.ContractDesc(K, Np, E, layout, reserved, D, u, out)


def status(d, rec=None):
    return lpx.contract_validate(d, rec)


def test_validate_accepts_well_formed():
    assert status(desc()) == lpx.OK
    for r in lpx.enumerate_records(3, 56, 1000, "dm", "bf16x3"):
        # (64, 11): D fragments + u ring + DOF-major output ring exceed LDS
        bad = ((64, 11),)
        want = lpx.ERR_UNSUPPORTED if (r.tile_e, r.prefetch) in bad else lpx.OK
        assert status(desc(layout=1), r) == want, lpx.describe(r)


@pytest.mark.parametrize("kw,code", [
    (dict(K=-1), lpx.ERR_INVALID_ARG),
    (dict(Np=-2), lpx.ERR_INVALID_ARG),
    (dict(E=-5), lpx.ERR_INVALID_ARG),
    (dict(layout=2), lpx.ERR_INVALID_ARG),
    (dict(reserved=1), lpx.ERR_INVALID_ARG),
    (dict(E=1 << 62), lpx.ERR_INVALID_ARG),          # K*E*Np overflows
    (dict(Np=129), lpx.ERR_UNSUPPORTED),
    (dict(D=None), lpx.ERR_INVALID_ARG),
    (dict(u=None), lpx.ERR_INVALID_ARG),
    (dict(out=None), lpx.ERR_INVALID_ARG),
    (dict(u=A + 8), lpx.ERR_INVALID_ARG),             # misaligned
    (dict(out=A + (1 << 24) + 4096), lpx.ERR_ALIAS),  # out overlaps u
    (dict(out=A), lpx.ERR_ALIAS),                      # out overlaps D
])
def test_validate_rejects(kw, code):
    assert status(desc(**kw)) == code
    assert lpx.last_error()


def test_zero_sizes_are_noops_even_with_null_pointers():
    for kw in (dict(E=0), dict(K=0), dict(Np=0)):
        d = desc(D=None, u=None, out=None, **kw)
        assert status(d) == lpx.OK
        # lpx_contract returns before any HIP call for a zero-size problem
        assert lpx.lib().lpx_contract(ctypes.byref(d), None, None) == lpx.OK


def test_assumption_checked():
    r = lpx.record("fp32", 32, 0, 1, assume_tile_divides=1)
    assert status(desc(E=1024), r) == lpx.OK
    assert status(desc(E=1000), r) == lpx.ERR_ASSUMPTION
    assert "assumes" in lpx.last_error()


def test_stacked_rows_limit():
    # the K operators are stacked into K*Np MFMA rows indexed with 32-bit
    # integers: K*Np beyond 2^31 - 16 is refused before any HIP call
    far = dict(u=A + (1 << 44), out=A + (1 << 45))  # D of 2^41 bytes does not overlap them
    assert status(desc(K=1 << 24, Np=128, **far)) == lpx.ERR_UNSUPPORTED  # 2^31 rows
    assert "stacked operator rows" in lpx.last_error()


@pytest.mark.parametrize("prec,Np,kmax", [
    # fp32: ceil(K*Np/16) row blocks * ceil(Np/4) k-steps * 64 lanes
    ("fp32", 128, (1 << 17) - 1),     # 2^14 fragments per operator
    ("fp32", 1, (1 << 29) - 16),      # one k-step, K/16 row blocks
    # bf16x3: ceil(Np/32) k-steps, two planes (hi, lo) in one index space
    ("bf16x3", 128, (1 << 19) - 1),   # 2^11 fragments per operator, x2 planes
    ("bf16", 128, (1 << 20) - 1),
])
def test_d_fragment_index_limit(prec, Np, kmax):
    # D's MFMA-order arrangement is indexed with 32-bit integers: problems
    # whose fragment count (times the planes) reaches 2^31 are refused before
    # any HIP call, for every record (validation only; no GPU run)
    far = dict(u=A + (1 << 44), out=A + (1 << 45))
    for pf in (0, 1, 2):
        rec = lpx.record(prec, 16, pf, 1)
        assert status(desc(K=kmax, Np=Np, E=16, **far), rec) in (lpx.OK, lpx.ERR_UNSUPPORTED)
        if pf == 0:
            assert status(desc(K=kmax, Np=Np, E=16, **far), rec) == lpx.OK
        assert status(desc(K=kmax + 16, Np=Np, E=16, **far), rec) == lpx.ERR_UNSUPPORTED
        assert "D fragments" in lpx.last_error()


def test_register_d_limits():
    # D in registers: fits Np <= 64 with ceil(K*Np/16) <= 12 row blocks
    assert status(desc(Np=56), lpx.record("fp32", 32, 4, 1)) == lpx.OK
    assert status(desc(Np=56), lpx.record("bf16x3", 32, 6, 1)) == lpx.OK
    assert status(desc(Np=84), lpx.record("fp32", 32, 4, 1)) == lpx.ERR_UNSUPPORTED
    assert status(desc(K=4, Np=56), lpx.record("fp32", 32, 4, 1)) == lpx.ERR_UNSUPPORTED
    assert status(desc(Np=56), lpx.record("fp32", 64, 6, 1)) == lpx.OK
    assert status(desc(Np=56), lpx.record("fp32", 64, 14, 1)) == lpx.OK
    assert status(desc(Np=56), lpx.record("fp32", 64, 4, 1)) == lpx.OK
    s, b = lpx.lds_bytes(3, 56, 1 << 20, "em", lpx.record("fp32", 32, 6, 1))
    assert s == lpx.OK and b == 4 * (32 * 64 + 32) * 4  # only the u ring


def test_lds_budget():
    # prefetch bit 0 stages all of D in LDS: Np = 128, K = 3 in FP32 needs
    # 24 row blocks * 32 k-steps * 64 lanes * 4 bytes, above 160 KiB
    r = lpx.record("fp32", 64, 1, 1)
    assert status(desc(Np=128), r) == lpx.ERR_UNSUPPORTED
    s, b = lpx.lds_bytes(3, 128, 4096, "em", r)
    assert s == lpx.ERR_UNSUPPORTED and b == 3 * 8 * 32 * 64 * 4
    # bit 1 alone stages only u: a four-slot ring, each slot a raw tile copy
    # with room for padding columns: 64 * 128 + 32 floats
    s, b = lpx.lds_bytes(3, 128, 4096, "em", lpx.record("fp32", 64, 2, 1))
    assert s == lpx.OK and b == 4 * (64 * 128 + 32) * 4
    # Np = 72 needs only 64 * 96 + 32 floats of tile, but the loader waves
    # write whole rounds of 64 chunks each: 4 waves * 8 rounds * 256 floats
    s, b = lpx.lds_bytes(3, 72, 4096, "em", lpx.record("fp32", 64, 2, 1))
    assert s == lpx.OK and b == 4 * (4 * 8 * 256) * 4
    # the full-scale shape fits both: the 3 stacked operators are 168 rows,
    # 11 row blocks of D (11*14*64*4 bytes) + ring 4*(64*64+32)*4
    s, b = lpx.lds_bytes(3, 56, 1 << 20, "em", lpx.record("fp32", 64, 3, 1))
    assert s == lpx.OK and b == 11 * 14 * 64 * 4 + 4 * (64 * 64 + 32) * 4
    # bf16x3: two bf16 planes of D fragments (16 B per lane each)
    s, b = lpx.lds_bytes(3, 56, 1 << 20, "em", lpx.record("bf16x3", 32, 3, 1))
    assert s == lpx.OK and b == 11 * 2 * 64 * 32 + 4 * (32 * 64 + 32) * 4
    s, b = lpx.lds_bytes(3, 56, 1 << 20, "em", lpx.record("fp32", 64, 0, 1))
    assert s == lpx.OK and b == 0
    # bit 3 adds a two-slot output ring: element-major K*tile_e*Np floats per
    # slot, DOF-major K*Np rows of tile_e + 4 floats
    s, b = lpx.lds_bytes(3, 56, 1 << 20, "em", lpx.record("fp32", 32, 14, 1))
    assert s == lpx.OK and b == 4 * (32 * 64 + 32) * 4 + 2 * 3 * 32 * 56 * 4
    s, b = lpx.lds_bytes(3, 56, 1 << 20, "dm", lpx.record("bf16x3", 32, 11, 1))
    assert s == lpx.OK and b == (11 * 2 * 64 * 32 + 4 * (32 * 64 + 32) * 4
                                 + 2 * 3 * 56 * 36 * 4)
    # K = 8 at Np = 120 with a 64-element tile: the output ring alone needs
    # 2*8*64*120*4 bytes
    s, b = lpx.lds_bytes(8, 120, 4096, "em", lpx.record("fp32", 64, 10, 1))
    assert s == lpx.ERR_UNSUPPORTED


def test_null_descriptor_and_split_args():
    L = lpx.lib()
    assert L.lpx_contract(None, None, None) == lpx.ERR_INVALID_ARG
    assert L.lpx_split_bf16(None, None, None, 0, None) == lpx.OK
    assert L.lpx_split_bf16(None, None, None, -1, None) == lpx.ERR_INVALID_ARG
    assert L.lpx_split_bf16(None, None, None, 10, None) == lpx.ERR_INVALID_ARG


def gdesc(M=256, N=256, K=256, A=A, lda=None, B=A + (1 << 24), ldb=None, C=A + (1 << 28), ldc=None):
    return lpx.GemmDesc(M, N, K, A, K if lda is None else lda, B, N if ldb is None else ldb,
                        C, N if ldc is None else ldc)


def test_gemm_validate():
    assert lpx.gemm_validate(gdesc()) == lpx.OK
    for prec in ("fp32", "bf16", "bf16x3"):
        for tiles in ((64, 64, 32), (128, 128, 64), (128, 64, 32)):
            assert lpx.gemm_validate(gdesc(), lpx.record(prec, gemm=tiles)) == lpx.OK
    assert lpx.gemm_validate(gdesc(), lpx.record("fp32", gemm=(256, 256, 32))) == lpx.OK
    for prec, tiles in (("bf16", (256, 256, 64)), ("bf16", (256, 128, 64)),
                        ("bf16x3", (256, 256, 32)), ("bf16x3", (256, 128, 32))):  # pre-split
        assert lpx.gemm_validate(gdesc(), lpx.record(prec, gemm=tiles)) == lpx.OK
    for prec, tiles in (("bf16x3", (128, 256, 32)), ("bf16x3", (256, 256, 64)),
                        ("fp32", (256, 256, 64)), ("bf16", (256, 128, 128))):
        assert lpx.gemm_validate(gdesc(), lpx.record(prec, gemm=tiles)) == lpx.ERR_UNSUPPORTED
    assert lpx.gemm_validate(gdesc(), lpx.record("fp32", gemm=(96, 64, 32))) == lpx.ERR_UNSUPPORTED
    assert lpx.gemm_validate(gdesc(M=-1)) == lpx.ERR_INVALID_ARG
    assert lpx.gemm_validate(gdesc(lda=100)) == lpx.ERR_INVALID_ARG   # below K
    assert lpx.gemm_validate(gdesc(lda=258)) == lpx.OK                # any lda >= K
    assert lpx.gemm_validate(gdesc(A=A + 4)) == lpx.ERR_INVALID_ARG   # misaligned
    assert lpx.gemm_validate(gdesc(C=A + 1024)) == lpx.ERR_ALIAS      # C overlaps A
    assert lpx.gemm_validate(gdesc(C=None)) == lpx.ERR_INVALID_ARG
    d = gdesc(M=0, A=None, B=None, C=None)
    assert lpx.gemm_validate(d) == lpx.OK
    assert lpx.lib().lpx_gemm(ctypes.byref(d), None, None) == lpx.OK   # no-op, no HIP call
    assert lpx.lib().lpx_gemm(None, None, None) == lpx.ERR_INVALID_ARG


def test_noalloc_refuses_oversize_arrangement_before_any_hip_call():
    # lpx_contract_noalloc keeps D's arrangement in a 1 MiB static scratch:
    # fp32 at Np = 128 takes ceil(K*128/16) * 32 * 64 * 4 bytes, 1 MiB at
    # K = 16; K = 17 is refused with no HIP call (none would work here)
    assert lpx.NOALLOC_SCRATCH_BYTES == 1 << 20
    far = dict(u=A + (1 << 44), out=A + (1 << 45))
    d = desc(K=17, Np=128, E=64, **far)
    assert status(d) == lpx.OK  # lpx_contract itself would take it
    assert lpx.contract_noalloc_status(d, None, stream=0) == lpx.ERR_UNSUPPORTED
    assert "scratch" in lpx.last_error()
    # bf16x3: 32-byte fragments, ceil(Np/32) steps: 8 * 4 * 64 * 32 bytes per
    # operator at Np = 128, 1 MiB at K = 16
    r = lpx.record("bf16x3", 32, 2, 1)
    assert lpx.contract_noalloc_status(desc(K=17, Np=128, E=64, **far), r, stream=0) == \
        lpx.ERR_UNSUPPORTED
    # invalid arguments are refused as lpx_contract refuses them
    assert lpx.contract_noalloc_status(desc(K=-1), None, stream=0) == lpx.ERR_INVALID_ARG
    # zero sizes are no-ops with no HIP call
    assert lpx.contract_noalloc_status(desc(E=0, D=None, u=None, out=None), None,
                                       stream=0) == lpx.OK


def dgdesc(K=3, Np=56, E=1000, layout=0, D=A, u=A + (1 << 24), G=A + (1 << 27),
           out=A + (1 << 28), reserved=0):
    return lpx.DgDesc(K, Np, E, layout, reserved, D, u, G, out)


def test_dg_volume_validation():
    st, rec = lpx.dg_volume_validate(dgdesc())
    assert st == lpx.OK and (rec.tile_e, rec.prefetch) == (64, 14)  # the NULL default
    for pf in (10, 11, 14):
        assert lpx.dg_volume_validate(dgdesc(), lpx.record("bf16x3", 32, pf, 1))[0] == lpx.OK
    for pf in (0, 1, 2, 3, 4, 6):  # no staged output tile: no epilogue
        assert lpx.dg_volume_validate(dgdesc(), lpx.record("fp32", 32, pf, 1))[0] == \
            lpx.ERR_UNSUPPORTED
        assert "staged output" in lpx.last_error()
    assert lpx.dg_volume_validate(dgdesc(K=4))[0] == lpx.ERR_UNSUPPORTED
    assert lpx.dg_volume_validate(dgdesc(G=None))[0] == lpx.ERR_INVALID_ARG
    assert lpx.dg_volume_validate(dgdesc(G=A + (1 << 27) + 4))[0] == lpx.ERR_INVALID_ARG
    assert lpx.dg_volume_validate(dgdesc(G=A + (1 << 28) + 64))[0] == lpx.ERR_ALIAS
    assert lpx.dg_volume_validate(dgdesc(out=A + 16))[0] == lpx.ERR_ALIAS  # out over D
    for kw in (dict(E=0), dict(K=0), dict(Np=0)):
        d = dgdesc(D=None, u=None, G=None, out=None, **kw)
        assert lpx.dg_volume_validate(d)[0] == lpx.OK
        assert lpx.lib().lpx_dg_volume(ctypes.byref(d), None, None) == lpx.OK
    # the default falls back to smaller tiles and D from memory where the
    # rings do not fit: Np = 120, DOF-major
    st, rec = lpx.dg_volume_validate(dgdesc(Np=120, layout=1, G=A + (1 << 30),
                                            out=A + (1 << 31)))
    assert st == lpx.OK and rec.prefetch == 10 and rec.tile_e < 64
    # the G area of the output slots counts against LDS: a record that fits
    # the plain contraction at the edge of the budget may not fit the dG one
    r = lpx.record("fp32", 64, 14, 1)
    s_plain, b_plain = lpx.lds_bytes(3, 56, 1000, "em", r)
    assert s_plain == lpx.OK


def cdesc(nt=100, ns=50, layout=0, tg=A, sr=A + (1 << 20), phi=A + (1 << 24), reserved=0):
    return lpx.CoulombDesc(nt, ns, layout, reserved, tg, sr, phi)


def test_coulomb_validation():
    v = lambda d, r=None: lpx.lib().lpx_coulomb_validate(  # noqa: E731
        ctypes.byref(d), ctypes.byref(r) if r is not None else None)
    assert v(cdesc()) == lpx.OK
    for rec in lpx.coulomb_records():
        assert v(cdesc(), rec) == lpx.OK
    assert len(lpx.coulomb_records()) == 18
    assert v(cdesc(), lpx.record("bf16x3", 16, 0, 1)) == lpx.ERR_UNSUPPORTED
    assert v(cdesc(), lpx.record("fp32", 16, 1, 1)) == lpx.ERR_UNSUPPORTED
    assert v(cdesc(), lpx.record("fp32", 16, 6, 1)) == lpx.ERR_UNSUPPORTED
    assert v(cdesc(tg=A + 4)) == lpx.ERR_INVALID_ARG          # AoS needs 16-byte records
    assert v(cdesc(layout=1, tg=A + 4)) == lpx.OK               # SoA: 4-byte floats
    assert v(cdesc(phi=A + 64)) == lpx.ERR_ALIAS
    assert v(cdesc(nt=-1)) == lpx.ERR_INVALID_ARG
    assert v(cdesc(layout=3)) == lpx.ERR_INVALID_ARG
    assert v(cdesc(sr=None)) == lpx.ERR_INVALID_ARG
    assert v(cdesc(ns=0, sr=None)) == lpx.OK
    d = cdesc(nt=0, tg=None, sr=None, phi=None)
    assert v(d) == lpx.OK and lpx.lib().lpx_coulomb(ctypes.byref(d), None, None) == lpx.OK


def sdesc(Np=56, nf=4, nfp=21, E=1000, layout=0, L=A, f=A + (1 << 20), s=A + (1 << 24),
          out=A + (1 << 26), reserved=0):
    return lpx.SurfaceDesc(Np, nf, nfp, layout, E, reserved, 0, L, f, s, out)


def test_dg_surface_validation():
    v = lambda d, r=None: lpx.lib().lpx_dg_surface_validate(  # noqa: E731
        ctypes.byref(d), ctypes.byref(r) if r is not None else None)
    assert v(sdesc()) == lpx.OK
    for prec in ("fp32", "bf16", "bf16x3"):
        for r in lpx.surface_records(prec):
            assert v(sdesc(), r) == lpx.OK
    assert v(sdesc(), lpx.record("fp32", 16, 0, 1)) == lpx.ERR_UNSUPPORTED  # not staged
    assert v(sdesc(), lpx.record("fp32", 16, 3, 1)) == lpx.ERR_UNSUPPORTED
    assert v(sdesc(Np=129)) == lpx.ERR_UNSUPPORTED
    # LDS: FP32 fragments nrb * ceil(M/4) * 256 bytes; Np = 128, M = 320 fits, 324 not
    assert v(sdesc(Np=128, nf=4, nfp=80)) == lpx.OK
    assert v(sdesc(Np=128, nf=4, nfp=81)) == lpx.ERR_UNSUPPORTED
    assert v(sdesc(f=A + (1 << 20) + 4)) == lpx.ERR_INVALID_ARG
    assert v(sdesc(out=A + (1 << 20) + 64)) == lpx.ERR_ALIAS
    assert v(sdesc(E=-1)) == lpx.ERR_INVALID_ARG
    assert v(sdesc(s=None)) == lpx.ERR_INVALID_ARG
    for kw in (dict(E=0), dict(Np=0), dict(nf=0)):
        d = sdesc(L=None, f=None, s=None, out=None, **kw)
        assert v(d) == lpx.OK and lpx.lib().lpx_dg_surface(ctypes.byref(d), None, None) == lpx.OK
