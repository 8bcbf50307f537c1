"""ctypes binding of liblpx (the C ABI in include/lpx.h).

Argument marshalling only: every step of the contraction runs in the HIP
kernels of liblpx.  PyTorch supplies device memory and streams.  There is no
fallback: if liblpx.so is missing or a call fails, an exception is raised.

torch is imported before liblpx.so is loaded, so that the library binds to the
HIP runtime torch already has in the process (one runtime, shared streams).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblpx.so")

# status codes (include/lpx.h)
OK = 0
MAX_RECORDS = 162  # LPX_MAX_RECORDS
ERR_INVALID_ARG = 1
ERR_UNSUPPORTED = 2
ERR_ASSUMPTION = 3
ERR_ALIAS = 4
ERR_HIP = 5
ERR_MODEL = 6
ERR_NOT_TUNED = 7
ERR_INTERNAL = 8

PRECISION = {"fp32": 0, "bf16": 1, "bf16x3": 2}
PRECISION_NAME = {v: k for k, v in PRECISION.items()}
LAYOUT = {"em": 0, "dm": 1}
NOALLOC_SCRATCH_BYTES = 1 << 20   # LPX_NOALLOC_SCRATCH_BYTES
RECORD_VERSION = 1


class LpxError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status


class Record(ctypes.Structure):
    """Transformation record (struct lpx_record)."""
    _fields_ = [
        ("version", ctypes.c_uint32),
        ("precision", ctypes.c_uint8),
        ("tile_e", ctypes.c_uint8),
        ("prefetch", ctypes.c_uint8),
        ("unroll", ctypes.c_uint8),
        ("assume_tile_divides", ctypes.c_uint8),
        ("order", ctypes.c_uint8),
        ("reserved0", ctypes.c_uint8 * 2),
        ("gemm_tm", ctypes.c_uint16),
        ("gemm_tn", ctypes.c_uint16),
        ("gemm_tk", ctypes.c_uint16),
        ("reserved1", ctypes.c_uint16),
    ]

    def key(self):
        return (self.precision, self.tile_e, self.prefetch, self.unroll,
                self.assume_tile_divides, self.order, self.gemm_tm, self.gemm_tn, self.gemm_tk)

    def __eq__(self, other):
        return isinstance(other, Record) and self.key() == other.key()

    def __hash__(self):
        return hash(self.key())

    def __repr__(self):
        return f"Record({describe(self)})"

    def as_dict(self):
        return {"precision": PRECISION_NAME[self.precision], "tile_e": self.tile_e,
                "prefetch": self.prefetch, "unroll": self.unroll,
                "assume_tile_divides": self.assume_tile_divides, "order": self.order,
                "gemm": [self.gemm_tm, self.gemm_tn, self.gemm_tk]}


class Problem(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("Np", ctypes.c_int32), ("E", ctypes.c_int64),
                ("layout", ctypes.c_int32), ("precision", ctypes.c_int32)]


class ContractDesc(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("Np", ctypes.c_int32), ("E", ctypes.c_int64),
                ("layout", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("D", ctypes.c_void_p), ("u", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class DgDesc(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("Np", ctypes.c_int32), ("E", ctypes.c_int64),
                ("layout", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("D", ctypes.c_void_p), ("u", ctypes.c_void_p), ("G", ctypes.c_void_p),
                ("out", ctypes.c_void_p)]


class SurfaceDesc(ctypes.Structure):
    _fields_ = [("Np", ctypes.c_int32), ("nf", ctypes.c_int32), ("nfp", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("E", ctypes.c_int64), ("reserved", ctypes.c_int32),
                ("reserved2", ctypes.c_int32), ("L", ctypes.c_void_p), ("f", ctypes.c_void_p),
                ("s", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class CoulombDesc(ctypes.Structure):
    _fields_ = [("nt", ctypes.c_int64), ("ns", ctypes.c_int64), ("layout", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("targets", ctypes.c_void_p),
                ("sources", ctypes.c_void_p), ("phi", ctypes.c_void_p)]


class GemmDesc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64)]


_lib = None


def lib():
    """The loaded liblpx.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1405_7470_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int32
        vp = ctypes.c_void_p
        L.lpx_version.restype = ctypes.c_char_p
        L.lpx_status_string.restype = ctypes.c_char_p
        L.lpx_status_string.argtypes = [st]
        L.lpx_last_error.restype = ctypes.c_char_p
        L.lpx_record_default.argtypes = [ctypes.c_int32, ctypes.POINTER(Record)]
        L.lpx_record_validate.argtypes = [ctypes.POINTER(Record)]
        L.lpx_record_describe.argtypes = [ctypes.POINTER(Record), ctypes.c_char_p, ctypes.c_size_t]
        L.lpx_record_enumerate.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Record),
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.lpx_contract_lds_bytes.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Record),
                                             ctypes.POINTER(ctypes.c_int64)]
        L.lpx_contract_validate.argtypes = [ctypes.POINTER(ContractDesc), ctypes.POINTER(Record)]
        L.lpx_contract.argtypes = [ctypes.POINTER(ContractDesc), ctypes.POINTER(Record), vp]
        L.lpx_contract_noalloc.argtypes = [ctypes.POINTER(ContractDesc), ctypes.POINTER(Record),
                                           vp]
        L.lpx_dg_volume.argtypes = [ctypes.POINTER(DgDesc), ctypes.POINTER(Record), vp]
        L.lpx_coulomb.argtypes = [ctypes.POINTER(CoulombDesc), ctypes.POINTER(Record), vp]
        L.lpx_dg_surface.argtypes = [ctypes.POINTER(SurfaceDesc), ctypes.POINTER(Record), vp]
        L.lpx_dg_surface_validate.argtypes = [ctypes.POINTER(SurfaceDesc), ctypes.POINTER(Record)]
        L.lpx_coulomb_validate.argtypes = [ctypes.POINTER(CoulombDesc), ctypes.POINTER(Record)]
        L.lpx_dg_volume_validate.argtypes = [ctypes.POINTER(DgDesc), ctypes.POINTER(Record),
                                             ctypes.POINTER(Record)]
        L.lpx_split_bf16.argtypes = [vp, vp, vp, ctypes.c_int64, vp]
        L.lpx_autotune.argtypes = [ctypes.POINTER(ContractDesc), ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, vp, ctypes.c_int64, vp, ctypes.POINTER(Record),
                                   ctypes.POINTER(ctypes.c_float), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)]
        f32p = ctypes.POINTER(ctypes.c_float)
        L.lpx_features.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Record), f32p]
        L.lpx_mlp_forward.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp]
        L.lpx_mlp_loss.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp]
        L.lpx_mlp_backward.argtypes = [vp, vp, vp, vp, ctypes.c_int32, vp, vp, vp]
        L.lpx_adam_step.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
        L.lpx_mlp_pick.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp]
        L.lpx_picker_save.argtypes = [ctypes.c_char_p, f32p, f32p, f32p]
        L.lpx_picker_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]
        L.lpx_picker_params.argtypes = [vp, f32p, f32p, f32p]
        L.lpx_picker_free.argtypes = [vp]
        L.lpx_pick_variant.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32, vp, vp,
                                       ctypes.POINTER(Record)]
        for name in ("lpx_features", "lpx_mlp_forward", "lpx_mlp_loss", "lpx_mlp_backward",
                     "lpx_adam_step", "lpx_mlp_pick", "lpx_picker_save", "lpx_picker_load",
                     "lpx_picker_params", "lpx_picker_free", "lpx_pick_variant"):
            getattr(L, name).restype = st
        L.lpx_tune_cache_insert.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Record)]
        L.lpx_tune_cache_clear.argtypes = []
        L.lpx_gemm.argtypes = [ctypes.POINTER(GemmDesc), ctypes.POINTER(Record), vp]
        L.lpx_gemm.restype = st
        L.lpx_gemm_validate.argtypes = [ctypes.POINTER(GemmDesc), ctypes.POINTER(Record)]
        L.lpx_gemm_validate.restype = st
        L.lpx_batch_submit.argtypes = [ctypes.POINTER(ContractDesc), ctypes.POINTER(Record),
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), vp]
        L.lpx_batch_submit.restype = st
        L.lpx_batch_tune.argtypes = [ctypes.POINTER(ContractDesc), ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, vp, ctypes.POINTER(Record)]
        L.lpx_batch_tune.restype = st
        L.lpx_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
        L.lpx_batch_info.restype = st
        L.lpx_batch_destroy.argtypes = [vp]
        L.lpx_batch_destroy.restype = st
        L.lpx_stream_probe.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp]
        L.lpx_stream_probe.restype = st
        for name in ("lpx_autotune", "lpx_tune_cache_insert", "lpx_tune_cache_clear",
                     "lpx_record_default", "lpx_record_validate", "lpx_record_describe",
                     "lpx_record_enumerate", "lpx_contract_lds_bytes", "lpx_contract_validate",
                     "lpx_contract", "lpx_contract_noalloc", "lpx_split_bf16",
                     "lpx_dg_volume", "lpx_dg_volume_validate", "lpx_coulomb",
                     "lpx_coulomb_validate", "lpx_dg_surface", "lpx_dg_surface_validate"):
            getattr(L, name).restype = st
        _lib = L
    return _lib


def _status_name(s):
    try:
        return lib().lpx_status_string(s).decode()
    except Exception:  # library not loadable: still report the number
        return f"status {s}"


def _check(status):
    if status != OK:
        raise LpxError(status, lib().lpx_last_error().decode())


def version() -> str:
    return lib().lpx_version().decode()


def last_error() -> str:
    return lib().lpx_last_error().decode()


# ------------------------------------------------------------------ records
def default_record(precision="fp32") -> Record:
    r = Record()
    _check(lib().lpx_record_default(PRECISION[precision], ctypes.byref(r)))
    return r


def record(precision="fp32", tile_e=16, prefetch=0, unroll=1, assume_tile_divides=0,
           gemm=(0, 0, 0), order=0) -> Record:
    r = default_record(precision)
    r.tile_e, r.prefetch, r.unroll = tile_e, prefetch, unroll
    r.assume_tile_divides = assume_tile_divides
    r.order = order
    r.gemm_tm, r.gemm_tn, r.gemm_tk = gemm
    return r


def validate_record(rec) -> int:
    return lib().lpx_record_validate(ctypes.byref(rec))


def describe(rec) -> str:
    buf = ctypes.create_string_buffer(160)
    s = lib().lpx_record_describe(ctypes.byref(rec), buf, len(buf))
    if s != OK:
        return f"<invalid record: {last_error()}>"
    return buf.value.decode()


def problem(K, Np, E, layout="em", precision="fp32") -> Problem:
    return Problem(K, Np, E, LAYOUT[layout], PRECISION[precision])


def enumerate_records(K, Np, E, layout="em", precision="fp32"):
    """Candidate records of a problem, in the library's canonical order."""
    p = problem(K, Np, E, layout, precision)
    n = ctypes.c_int32()
    _check(lib().lpx_record_enumerate(ctypes.byref(p), None, 0, ctypes.byref(n)))
    arr = (Record * n.value)()
    _check(lib().lpx_record_enumerate(ctypes.byref(p), arr, n.value, ctypes.byref(n)))
    return list(arr)


def lds_bytes(K, Np, E, layout, rec):
    """(status, bytes) of dynamic LDS per work-group for the record."""
    p = problem(K, Np, E, layout, PRECISION_NAME[rec.precision])
    b = ctypes.c_int64()
    s = lib().lpx_contract_lds_bytes(ctypes.byref(p), ctypes.byref(rec), ctypes.byref(b))
    return s, b.value


# -------------------------------------------------------------- contraction
def _stream_handle(stream):
    """hipStream_t of a torch stream (None = torch's current stream; 0 = the
    null stream)."""
    if isinstance(stream, int):
        return ctypes.c_void_p(stream or None)
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def contract_shapes(D, u, layout):
    K, Np, Np2 = D.shape
    if Np != Np2:
        raise ValueError(f"D must be (K, Np, Np), got {tuple(D.shape)}")
    if u.dim() != 2:
        raise ValueError("u must be 2-D")
    if layout == "em":
        E = u.shape[0]
        if u.shape[1] != Np:
            raise ValueError(f"element-major u must be (E, {Np}), got {tuple(u.shape)}")
    elif layout == "dm":
        E = u.shape[1]
        if u.shape[0] != Np:
            raise ValueError(f"DOF-major u must be ({Np}, E), got {tuple(u.shape)}")
    else:
        raise ValueError(f"unknown layout {layout!r}")
    return K, Np, E


def make_desc(D, u, out, layout):
    K, Np, E = contract_shapes(D, u, layout)
    for name, t in (("D", D), ("u", u), ("out", out)):
        if t.dtype != torch.float32:
            raise TypeError(f"{name} must be float32")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    if out.numel() != K * E * Np:
        raise ValueError(f"out must hold K*E*Np = {K * E * Np} floats")
    return ContractDesc(K, Np, E, LAYOUT[layout], 0, D.data_ptr() if D.numel() else None,
                        u.data_ptr() if u.numel() else None,
                        out.data_ptr() if out.numel() else None)


def out_shape(K, Np, E, layout):
    return (K, E, Np) if layout == "em" else (K, Np, E)


def contract(D, u, out=None, layout="em", record=None, stream=None):
    """out[k,e,i] = sum_j D[k][i][j] u[e][j] on the GPU through lpx_contract.

    D: (K, Np, Np) float32 CUDA tensor.  u: (E, Np) for layout "em", (Np, E)
    for "dm".  out (allocated if None): (K, E, Np) for "em", (K, Np, E) for
    "dm".  record: a Record (None = the untuned FP32 default).
    """
    K, Np, E = contract_shapes(D, u, layout)
    if out is None:
        out = torch.empty(out_shape(K, Np, E, layout), dtype=torch.float32, device=u.device)
    desc = make_desc(D, u, out, layout)
    recp = ctypes.byref(record) if record is not None else None
    _check(lib().lpx_contract(ctypes.byref(desc), recp, _stream_handle(stream)))
    return out


def surface_desc(L, f, s, out, nf, layout="em"):
    """Descriptor of the dG surface (lift) term from CUDA tensors: L (Np, M);
    f (E, M) and s (E, nf) for "em", (M, E) and (nf, E) for "dm"; out like
    f with Np in place of M."""
    Np, M = L.shape
    if nf <= 0 or M % nf:
        raise ValueError("nf must divide the operator's column count")
    E = f.shape[0] if layout == "em" else f.shape[1]
    want = {"f": (E, M) if layout == "em" else (M, E), "s": (E, nf) if layout == "em" else (nf, E),
            "out": (E, Np) if layout == "em" else (Np, E)}
    for name, t in (("L", L), ("f", f), ("s", s), ("out", out)):
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float32 tensor")
        if name in want and tuple(t.shape) != want[name]:
            raise ValueError(f"{name} must have shape {want[name]}")
    ptr = lambda t: t.data_ptr() if t.numel() else None  # noqa: E731
    return SurfaceDesc(Np, nf, M // nf, LAYOUT[layout], E, 0, 0, ptr(L), ptr(f), ptr(s), ptr(out))


def dg_surface(L, f, s, nf, out=None, layout="em", record=None, stream=None):
    """out[e,i] = sum_m L[i][m] s(e, m // nfp) f(e, m) through lpx_dg_surface."""
    Np = L.shape[0]
    E = f.shape[0] if layout == "em" else f.shape[1]
    if out is None:
        out = torch.empty((E, Np) if layout == "em" else (Np, E), dtype=torch.float32,
                          device=f.device)
    d = surface_desc(L, f, s, out, nf, layout)
    recp = ctypes.byref(record) if record is not None else None
    _check(lib().lpx_dg_surface(ctypes.byref(d), recp, _stream_handle(stream)))
    return out


def surface_records(precision="fp32"):
    """The lift variants of a precision: 1, 2 or 4 element blocks per wave."""
    return [record(precision, t, 1, 1) for t in (16, 32, 64)]


def coulomb_desc(targets, sources, phi, layout="em"):
    """Descriptor of the Coulomb potential from CUDA tensors: AoS ("em")
    targets (nt, 4), sources (ns, 4); SoA ("dm") targets (3, nt), sources
    (4, ns); phi (nt,)."""
    if layout == "em":
        nt, ns = targets.shape[0], sources.shape[0]
        ok = targets.dim() == 2 and targets.shape[1] == 4 and sources.shape[1:] == (4,)
    else:
        nt, ns = targets.shape[1], sources.shape[1]
        ok = targets.dim() == 2 and targets.shape[0] == 3 and sources.shape[0] == 4
    if not ok:
        raise ValueError("targets/sources shapes do not match the layout")
    for name, t in (("targets", targets), ("sources", sources), ("phi", phi)):
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float32 tensor")
    if phi.numel() != nt:
        raise ValueError("phi must hold nt floats")
    ptr = lambda t: t.data_ptr() if t.numel() else None  # noqa: E731
    return CoulombDesc(nt, ns, LAYOUT[layout], 0, ptr(targets), ptr(sources), ptr(phi))


def coulomb(targets, sources, phi=None, layout="em", record=None, stream=None):
    """phi[t] = sum_s q_s / |x_t - y_s| through lpx_coulomb."""
    nt = targets.shape[0] if layout == "em" else targets.shape[1]
    if phi is None:
        phi = torch.empty(nt, dtype=torch.float32, device=targets.device)
    d = coulomb_desc(targets, sources, phi, layout)
    recp = ctypes.byref(record) if record is not None else None
    _check(lib().lpx_coulomb(ctypes.byref(d), recp, _stream_handle(stream)))
    return phi


def coulomb_records():
    """The Coulomb variants: source tile 256/512/1024 (tile_e 16/32/64),
    sources staged in LDS or not (prefetch 2/0), 1/2/4 targets per thread."""
    return [record("fp32", t, p, u) for t in (16, 32, 64) for p in (0, 2) for u in (1, 2, 4)]


def g_shape(K, E, layout):
    """Shape of the geometric factors of the dG volume term."""
    return (E, K, K) if layout == "em" else (K, K, E)


def make_dg_desc(D, u, G, out, layout):
    K, Np, E = contract_shapes(D, u, layout)
    for name, t in (("D", D), ("u", u), ("G", G), ("out", out)):
        if t.dtype != torch.float32:
            raise TypeError(f"{name} must be float32")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    if tuple(G.shape) != g_shape(K, E, layout):
        raise ValueError(f"G must have shape {g_shape(K, E, layout)}")
    if out.numel() != K * E * Np:
        raise ValueError(f"out must hold K*E*Np = {K * E * Np} floats")
    ptr = lambda t: t.data_ptr() if t.numel() else None  # noqa: E731
    return DgDesc(K, Np, E, LAYOUT[layout], 0, ptr(D), ptr(u), ptr(G), ptr(out))


def dg_volume(D, u, G, out=None, layout="em", record=None, stream=None):
    """dG volume term out[d,e,i] = sum_k G(e,d,k) sum_j D[k][i][j] u[e][j]
    through lpx_dg_volume.  G: (E, K, K) for "em", (K, K, E) for "dm"; out
    as for contract().  record: a staged-output Record (prefetch 10, 11 or
    14) or None (the library's default for the shape)."""
    K, Np, E = contract_shapes(D, u, layout)
    if out is None:
        out = torch.empty(out_shape(K, Np, E, layout), dtype=torch.float32, device=u.device)
    desc = make_dg_desc(D, u, G, out, layout)
    recp = ctypes.byref(record) if record is not None else None
    _check(lib().lpx_dg_volume(ctypes.byref(desc), recp, _stream_handle(stream)))
    return out


def dg_volume_validate(desc, rec=None):
    """(status, record used) of lpx_dg_volume_validate."""
    chosen = Record()
    recp = ctypes.byref(rec) if rec is not None else None
    st = lib().lpx_dg_volume_validate(ctypes.byref(desc), recp, ctypes.byref(chosen))
    return st, chosen


def contract_noalloc(D, u, out, layout="em", record=None, stream=None):
    """The same contraction through lpx_contract_noalloc, which allocates
    nothing (D's arrangement, when the record needs one, goes to the
    library's static device scratch).  `out` must be given."""
    K, Np, E = contract_shapes(D, u, layout)
    desc = make_desc(D, u, out, layout)
    recp = ctypes.byref(record) if record is not None else None
    _check(lib().lpx_contract_noalloc(ctypes.byref(desc), recp, _stream_handle(stream)))
    return out


def contract_noalloc_status(desc, rec=None, stream=None) -> int:
    """Raw status of lpx_contract_noalloc (for tests of its refusals)."""
    recp = ctypes.byref(rec) if rec is not None else None
    return lib().lpx_contract_noalloc(ctypes.byref(desc), recp, _stream_handle(stream))


def contract_validate(desc, rec=None) -> int:
    """Status lpx_contract would return for (desc, rec) before any launch."""
    recp = ctypes.byref(rec) if rec is not None else None
    return lib().lpx_contract_validate(ctypes.byref(desc), recp)


def split_bf16(x, hi=None, lo=None, stream=None):
    """(hi, lo) raw bfloat16 bit patterns (int16 tensors) of an fp32 tensor."""
    if x.dtype != torch.float32 or not x.is_contiguous():
        raise TypeError("x must be a contiguous float32 tensor")
    if hi is None:
        hi = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    if lo is None:
        lo = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    n = x.numel()
    _check(lib().lpx_split_bf16(ctypes.c_void_p(x.data_ptr() if n else None),
                                ctypes.c_void_p(hi.data_ptr() if n else None),
                                ctypes.c_void_p(lo.data_ptr() if n else None), n,
                                _stream_handle(stream)))
    return hi, lo


# ------------------------------------------------------------- autotuning
def autotune(D, u, out=None, layout="em", precision="fp32", warmup=2, reps=7, stream=None,
             flush=None):
    """Exhaustive tuning on the given buffers; returns (best Record, list of
    median microseconds per candidate in enumeration order; inf = skipped).
    flush: optional CUDA tensor overwritten before every timed launch."""
    K, Np, E = contract_shapes(D, u, layout)
    if out is None:
        out = torch.empty(out_shape(K, Np, E, layout), dtype=torch.float32, device=u.device)
    desc = make_desc(D, u, out, layout)
    best = Record()
    times = (ctypes.c_float * MAX_RECORDS)()
    n = ctypes.c_int32()
    fptr = ctypes.c_void_p(flush.data_ptr()) if flush is not None else None
    fbytes = flush.numel() * flush.element_size() if flush is not None else 0
    _check(lib().lpx_autotune(ctypes.byref(desc), PRECISION[precision], warmup, reps,
                              fptr, fbytes, _stream_handle(stream), ctypes.byref(best), times,
                              MAX_RECORDS, ctypes.byref(n)))
    return best, [times[i] for i in range(n.value)]


def tune_cache_insert(K, Np, E, layout, rec):
    p = problem(K, Np, E, layout, PRECISION_NAME[rec.precision])
    _check(lib().lpx_tune_cache_insert(ctypes.byref(p), ctypes.byref(rec)))


def tune_cache_clear():
    _check(lib().lpx_tune_cache_clear())


def stream_probe(x, y, fanout=1, stream=None):
    """y[r*n:(r+1)*n] = x for r < fanout (HBM streaming probe)."""
    n = x.numel()
    if y.numel() != fanout * n:
        raise ValueError("y must hold fanout * x.numel() floats")
    _check(lib().lpx_stream_probe(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                  n, fanout, _stream_handle(stream)))
    return y


# -------------------------------------------------------------------- GEMM
def gemm(A, B, C=None, record=None, stream=None):
    """C = A @ B (row-major float32 CUDA tensors) through lpx_gemm."""
    if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("A (M, K) and B (K, N) expected")
    M, K = A.shape
    N = B.shape[1]
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    for name, t in (("A", A), ("B", B), ("C", C)):
        if t.dtype != torch.float32 or t.stride(1) != 1:
            raise ValueError(f"{name} must be float32 with unit column stride")
    d = GemmDesc(M, N, K, A.data_ptr() if A.numel() else None, A.stride(0) if M else K,
                 B.data_ptr() if B.numel() else None, B.stride(0) if K else N,
                 C.data_ptr() if C.numel() else None, C.stride(0) if M else N)
    recp = ctypes.byref(record) if record is not None else None
    _check(lib().lpx_gemm(ctypes.byref(d), recp, _stream_handle(stream)))
    return C


def gemm_validate(desc, rec=None) -> int:
    recp = ctypes.byref(rec) if rec is not None else None
    return lib().lpx_gemm_validate(ctypes.byref(desc), recp)


# ------------------------------------------------------------ ragged batch
class Batch:
    """A ragged batch of contractions replayed as one graph: one persistent
    launch per kernel the instances' records select.

    items: list of (D, u, out, layout) CUDA tensors; records: list of Record
    (one per item, each honoured) or None (tuning cache / default).
    submit() replays, optionally with new tensors of the same shapes."""

    def __init__(self, items, records=None, stream=None):
        self.handle = ctypes.c_void_p(None)
        self.n = len(items)
        self._submit(items, records, stream)

    def _descs(self, items):
        arr = (ContractDesc * len(items))()
        for i, (D, u, out, layout) in enumerate(items):
            arr[i] = make_desc(D, u, out, layout)
        return arr

    def _submit(self, items, records, stream):
        descs = self._descs(items)
        recs = None
        if records is not None:
            recs = (Record * len(records))(*records)
        _check(lib().lpx_batch_submit(descs, recs, len(items), ctypes.byref(self.handle),
                                      _stream_handle(stream)))
        self._keep = items  # the caller's tensors stay referenced until the next submit

    def submit(self, items=None, stream=None):
        """Replays the graph; with items, first points it at new tensors of
        the same shapes."""
        if items is None:
            _check(lib().lpx_batch_submit(None, None, self.n, ctypes.byref(self.handle),
                                          _stream_handle(stream)))
            return
        self._submit(items, None, stream)

    def info(self):
        t, te, g, l = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().lpx_batch_info(self.handle, ctypes.byref(t), ctypes.byref(te), ctypes.byref(g),
                                    ctypes.byref(l)))
        return {"tiles": t.value, "kernels": te.value, "grid": g.value, "lds_bytes": l.value}

    def destroy(self):
        if self.handle:
            torch.cuda.synchronize()
            lib().lpx_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def batch_tune(items, precision="fp32", warmup=1, reps=5, stream=None):
    """Records for a batch of (D, u, out, layout) items from timing each
    (K, Np, layout) group as a batch (lpx_batch_tune); one Record per item.
    Overwrites every out tensor."""
    arr = (ContractDesc * len(items))()
    for i, (D, u, out, layout) in enumerate(items):
        arr[i] = make_desc(D, u, out, layout)
    recs = (Record * len(items))()
    _check(lib().lpx_batch_tune(arr, len(items), PRECISION[precision], warmup, reps,
                                _stream_handle(stream), recs))
    return list(recs)


# ------------------------------------------------------------ cost model
MLP_FEATURES, MLP_HIDDEN, MLP_PARAMS = 13, 64, 5121
PICK_UNTUNED, PICK_EXHAUSTIVE, PICK_LEARNED = 0, 1, 2


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def features(K, Np, E, layout, rec):
    """The 12 cost-model features of (problem, record) as a list."""
    p = problem(K, Np, E, layout, PRECISION_NAME[rec.precision])
    out = (ctypes.c_float * MLP_FEATURES)()
    _check(lib().lpx_features(ctypes.byref(p), ctypes.byref(rec), out))
    return list(out)


def mlp_forward(params, X, act=None, y=None, stream=None):
    n = X.shape[0]
    if y is None:
        y = torch.empty(n, device=X.device)
    _check(lib().lpx_mlp_forward(_ptr(params), _ptr(X), n, _ptr(act), _ptr(y), _stream_handle(stream)))
    return y


def mlp_loss(y, t, dy=None, loss=None, stream=None):
    n = y.shape[0]
    if dy is None:
        dy = torch.empty(n, device=y.device)
    if loss is None:
        loss = torch.empty(1, device=y.device)
    _check(lib().lpx_mlp_loss(_ptr(y), _ptr(t), n, _ptr(dy), _ptr(loss), _stream_handle(stream)))
    return dy, loss


def mlp_backward(params, X, act, dy, grads=None, work=None, stream=None):
    n = X.shape[0]
    if grads is None:
        grads = torch.empty(MLP_PARAMS, device=X.device)
    if work is None:
        work = torch.empty((max(n, 1), 2 * MLP_HIDDEN), device=X.device)
    _check(lib().lpx_mlp_backward(_ptr(params), _ptr(X), _ptr(act), _ptr(dy), n, _ptr(work),
                                  _ptr(grads), _stream_handle(stream)))
    return grads


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().lpx_adam_step(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.numel(), step,
                               lr, beta1, beta2, eps, _stream_handle(stream)))


def mlp_pick(params, feats, mean, std, pred=None, best=None, stream=None):
    n = feats.shape[0]
    if best is None:
        best = torch.empty(1, dtype=torch.int32, device=feats.device)
    _check(lib().lpx_mlp_pick(_ptr(params), _ptr(feats), n, _ptr(mean), _ptr(std), _ptr(pred),
                              _ptr(best), _stream_handle(stream)))
    return best


def picker_save(path, params, mean, std):
    import numpy as np
    arr = [np.ascontiguousarray(a, dtype=np.float32) for a in (params, mean, std)]
    fp = ctypes.POINTER(ctypes.c_float)
    _check(lib().lpx_picker_save(str(path).encode(), *[a.ctypes.data_as(fp) for a in arr]))


class Picker:
    """A loaded cost model (lpx_picker_load); raises LpxError(ERR_MODEL) on a
    missing or corrupt file."""

    def __init__(self, path):
        self.handle = ctypes.c_void_p(None)
        _check(lib().lpx_picker_load(str(path).encode(), ctypes.byref(self.handle)))

    def params(self):
        import numpy as np
        p = np.empty(MLP_PARAMS, np.float32)
        m = np.empty(MLP_FEATURES, np.float32)
        s = np.empty(MLP_FEATURES, np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        _check(lib().lpx_picker_params(self.handle, p.ctypes.data_as(fp), m.ctypes.data_as(fp),
                                       s.ctypes.data_as(fp)))
        return p, m, s

    def close(self):
        if self.handle:
            lib().lpx_picker_free(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pick_variant(K, Np, E, layout, precision, mode=PICK_LEARNED, picker=None, stream=None):
    """Record chosen for the problem by mode (untuned / exhaustive / learned)."""
    p = problem(K, Np, E, layout, precision)
    out = Record()
    h = picker.handle if picker is not None else None
    _check(lib().lpx_pick_variant(ctypes.byref(p), mode, h, _stream_handle(stream),
                                  ctypes.byref(out)))
    return out
