"""Python binding of libstats.so -- single-pass sufficient statistics on MI355X.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/stats.h``; the names below are
the C entry points.  Device memory and streams come from the caller (for
example PyTorch tensors and ``torch.cuda.current_stream().cuda_stream``) as
plain integer addresses.

If ``libstats.so`` has not been built this module raises on import: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstats.so")

try:  # share the process's HIP runtime with PyTorch when it is present
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2604_23826_amd/build.py "
                      "(the statistics path has no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

# ---- constants (include/stats.h) ---------------------------------------------
STATS_MAX_P = 1024
STATS_MAX_PLANES = 32
STATS_MASK_WORDS = STATS_MAX_P // 64
STATS_OK, STATS_E_ARG, STATS_E_STATE, STATS_E_HIP, STATS_E_NOMEM = 0, -1, -2, -3, -4
STATS_E_INEXACT, STATS_E_PARSE, STATS_E_MISMATCH, STATS_E_IO = -5, -6, -7, -8
STATS_I32, STATS_I64, STATS_F32, STATS_F64 = 1, 2, 3, 4
STATS_COL_INTEGER, STATS_COL_IDENTIFIER = 1, 2
STATS_MEM_DEVICE, STATS_MEM_HOST_PINNED, STATS_MEM_HOST = 0, 1, 2
STATS_PREC_FP64, STATS_PREC_SPLIT, STATS_PREC_AUTO = 0, 1, 2
STATS_PREC_SPLIT_BF16 = STATS_PREC_SPLIT  # former name
STATS_CFG_TIMING = 1
STATS_CFG_PAIRWISE = 2
STATS_NOALLOC_SCRATCH_BYTES = 8 << 20
(STATS_K_ACCUM, STATS_K_MERGE, STATS_K_FINALIZE, STATS_K_SYRK, STATS_K_SEGMENTED,
 STATS_K_TEXT, STATS_K_COPY, STATS_K_COUNT) = range(8)

DTYPE_CODE = {np.dtype(np.int32): STATS_I32, np.dtype(np.int64): STATS_I64,
              np.dtype(np.float32): STATS_F32, np.dtype(np.float64): STATS_F64}
ELEM_SIZE = {STATS_I32: 4, STATS_I64: 8, STATS_F32: 4, STATS_F64: 8}


class Column(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("plane", ctypes.c_int32),
                ("byte_offset", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Config(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("cols", ctypes.POINTER(Column)),
                ("n_planes", ctypes.c_int32), ("row_stride", ctypes.c_int64 * STATS_MAX_PLANES),
                ("precision", ctypes.c_int32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("staging_rows", ctypes.c_int64),
                ("block_rows", ctypes.c_int64), ("flags", ctypes.c_uint32)]


class FinalizeOpts(ctypes.Structure):
    _fields_ = [("column_mask", ctypes.c_uint64 * STATS_MASK_WORDS), ("ddof", ctypes.c_int32),
                ("pca_on", ctypes.c_int32), ("want_vectors", ctypes.c_int32)]


class I128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_int64)]


_vp, _i32, _i64, _u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
_sig = {
    "stats_open": [ctypes.POINTER(Config), ctypes.POINTER(_vp)],
    "stats_open_groups": [ctypes.POINTER(Config), _i32, ctypes.POINTER(_vp)],
    "stats_accumulate": [_vp, _vp, _i64, _i32],
    "stats_accumulate_noalloc": [_vp, _vp, _i64],
    "stats_accumulate_file": [_vp, ctypes.c_char_p, _i64, _i64],
    "stats_finalize_pairwise": [_vp, _i32, _vp, _vp, _vp, _vp],
    "stats_text_to_binary": [_vp, _vp, _i64, _i32, _i32, _vp, _i64, ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
    "stats_accumulate_text": [_vp, _vp, _i64, _i32, _i32, ctypes.POINTER(_i64)],
    "stats_accumulate_segmented": [_vp, _vp, _vp, _i32],
    "stats_merge": [_vp, _vp],
    "stats_sync": [_vp],
    "stats_reset": [_vp],
    "stats_raw": [_vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "stats_finalize": [_vp, ctypes.POINTER(FinalizeOpts), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "stats_finalize_groups": [_vp, ctypes.POINTER(FinalizeOpts), _vp, _vp, _vp, _vp],
    "stats_group_raw": [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp],
    "stats_serialize": [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)],
    "stats_deserialize": [_vp, ctypes.c_size_t, ctypes.POINTER(Config), ctypes.POINTER(_vp)],
    "stats_kernel_time": [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double)],
    "stats_read_probe": [_vp, _vp, _i32, _vp, ctypes.POINTER(ctypes.c_double)],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.stats_close.argtypes = [_vp]
_lib.stats_close.restype = None
_lib.stats_last_error.argtypes = []
_lib.stats_last_error.restype = ctypes.c_char_p


class StatsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"stats error {code}: {msg}")
        self.code = code
        self.msg = msg


def stats_last_error() -> str:
    return _lib.stats_last_error().decode()


def _check(rc: int) -> None:
    if rc != STATS_OK:
        raise StatsError(rc, stats_last_error())


def _ptr(x) -> int:
    """Address of a numpy array, a torch tensor or an int."""
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    raise TypeError(f"cannot take the address of {type(x)}")


def make_config(columns, row_strides, device: int = 0, stream=None, precision: int = STATS_PREC_AUTO,
                block_rows: int = 0, staging_rows: int = 0, timing: bool = False,
                pairwise: bool = False) -> Config:
    """columns: list of (dtype_code, plane, byte_offset, flags)."""
    cols = (Column * len(columns))(*[Column(*c) for c in columns])
    cfg = Config()
    cfg.p = len(columns)
    cfg.cols = ctypes.cast(cols, ctypes.POINTER(Column))
    cfg._cols_keepalive = cols
    cfg.n_planes = len(row_strides)
    for k, s in enumerate(row_strides):
        cfg.row_stride[k] = int(s)
    cfg.precision = precision
    cfg.device = device
    cfg.stream = stream
    cfg.staging_rows = staging_rows
    cfg.block_rows = block_rows
    cfg.flags = (STATS_CFG_TIMING if timing else 0) | (STATS_CFG_PAIRWISE if pairwise else 0)
    return cfg


def stats_open(cfg: Config) -> int:
    h = _vp()
    _check(_lib.stats_open(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def stats_open_groups(cfg: Config, ngroups: int) -> int:
    h = _vp()
    _check(_lib.stats_open_groups(ctypes.byref(cfg), ngroups, ctypes.byref(h)))
    return h.value


# Device tensors handed to a call that returns before its kernels have read
# them: the handle's work is ordered on its own stream, which torch's caching
# allocator does not know of, so a temporary freed on return could be handed
# out again (and overwritten) while still being read.  The binding keeps them
# referenced until the next call that waits for the handle's stream (sync,
# raw, finalize, serialize, close) -- the lifetime the C interface asks of
# its callers.
_held: dict = {}


def _hold(h: int, objs) -> None:
    keep = [o for o in objs if hasattr(o, "data_ptr")]
    if keep:
        _held.setdefault(h, []).extend(keep)


def _release(h: int) -> None:
    _held.pop(h, None)


def _planes(planes):
    arr = (_vp * STATS_MAX_PLANES)()
    for k, p in enumerate(planes):
        arr[k] = _ptr(p)
    return arr


def stats_accumulate(h: int, planes, nrows: int, mem_kind: int = STATS_MEM_DEVICE) -> None:
    _check(_lib.stats_accumulate(h, _planes(planes), nrows, mem_kind))
    _hold(h, planes)


def stats_accumulate_noalloc(h: int, planes, nrows: int) -> None:
    """Device input, p <= 16, no allocation in the call (see stats.h)."""
    _check(_lib.stats_accumulate_noalloc(h, _planes(planes), nrows))
    _hold(h, planes)


def stats_accumulate_file(h: int, path: str, offset: int, nrows: int) -> None:
    """Fixed-width records of a file (one-plane handle; see stats.h)."""
    _check(_lib.stats_accumulate_file(h, os.fsencode(path), offset, nrows))


def stats_finalize_pairwise(h: int, p: int, ddof: int = 1) -> dict:
    """n, mean, cov, corr of a pairwise (missing-value) handle (see stats.h)."""
    n = np.zeros((p, p), dtype=np.int64)
    mean = np.zeros(p)
    cov = np.zeros((p, p))
    corr = np.zeros((p, p))
    _check(_lib.stats_finalize_pairwise(h, ddof, n.ctypes.data, mean.ctypes.data, cov.ctypes.data,
                                        corr.ctypes.data))
    _release(h)
    return {"n": n, "mean": mean, "cov": cov, "corr": corr}


def stats_text_to_binary(h: int, buf, nbytes: int, out_planes, max_rows: int,
                         mem_kind: int = STATS_MEM_DEVICE, is_last: bool = False):
    """(rows written, bytes consumed) of a CSV chunk converted on the GPU into
    the handle's binary layout (see stats.h)."""
    rows, used = _i64(0), _i64(0)
    _check(_lib.stats_text_to_binary(h, _ptr(buf), nbytes, mem_kind, 1 if is_last else 0,
                                     _planes(out_planes), max_rows, ctypes.byref(rows), ctypes.byref(used)))
    return rows.value, used.value


def stats_accumulate_text(h: int, buf, nbytes: int, mem_kind: int = STATS_MEM_DEVICE,
                          is_last: bool = False) -> int:
    used = _i64(0)
    _check(_lib.stats_accumulate_text(h, _ptr(buf), nbytes, mem_kind, 1 if is_last else 0,
                                      ctypes.byref(used)))
    _hold(h, [buf])
    return used.value


def stats_accumulate_segmented(h: int, planes, row_offsets: np.ndarray,
                               mem_kind: int = STATS_MEM_DEVICE) -> None:
    off = np.ascontiguousarray(row_offsets, dtype=np.int64)
    _check(_lib.stats_accumulate_segmented(h, _planes(planes), off.ctypes.data, mem_kind))
    _hold(h, planes)


def stats_merge(dst: int, src: int) -> None:
    _check(_lib.stats_merge(dst, src))


def stats_sync(h: int) -> None:
    _check(_lib.stats_sync(h))
    _release(h)


def stats_reset(h: int) -> None:
    _check(_lib.stats_reset(h))


def _i128_to_int(v: I128) -> int:
    return (int(v.hi) << 64) | int(v.lo)


def _raw_outputs(p):
    return {"n": _i64(0), "s_int": (I128 * p)(), "s_f64": np.zeros(p),
            "C_int": (I128 * (p * p))(), "C_f64": np.zeros((p, p)),
            "exact": np.zeros((p, p), dtype=np.uint8)}


def _raw_result(o, p):
    return {"n": o["n"].value, "s_int": [_i128_to_int(o["s_int"][i]) for i in range(p)],
            "s_f64": o["s_f64"],
            "C_int": [[_i128_to_int(o["C_int"][i * p + j]) for j in range(p)] for i in range(p)],
            "C_f64": o["C_f64"], "exact": o["exact"].astype(bool)}


def stats_raw(h: int, p: int) -> dict:
    """(N, s, C): exact Python ints where exact, FP64 for every entry."""
    o = _raw_outputs(p)
    _check(_lib.stats_raw(h, ctypes.byref(o["n"]), o["s_int"], o["s_f64"].ctypes.data, o["C_int"],
                          o["C_f64"].ctypes.data, o["exact"].ctypes.data))
    _release(h)
    return _raw_result(o, p)


def stats_group_raw(h: int, g: int, p: int) -> dict:
    o = _raw_outputs(p)
    _check(_lib.stats_group_raw(h, g, ctypes.byref(o["n"]), o["s_int"], o["s_f64"].ctypes.data,
                                o["C_int"], o["C_f64"].ctypes.data, o["exact"].ctypes.data))
    _release(h)
    return _raw_result(o, p)


def finalize_opts(mask=None, ddof: int = 1, pca_on: int = 0, want_vectors: int = 1) -> FinalizeOpts:
    o = FinalizeOpts()
    if mask is not None:
        for c in mask:
            o.column_mask[c // 64] |= 1 << (c % 64)
    o.ddof = ddof
    o.pca_on = pca_on
    o.want_vectors = want_vectors
    return o


def stats_finalize(h: int, p: int, mask=None, ddof: int = 1, pca_on: int = 0,
                   want_vectors: int = 1) -> dict:
    """Means, cov, corr and PCA of the kept columns (p' of them; flat C arrays
    of p' x p' are reshaped here).  With want_vectors=0 the library leaves
    eigvec unwritten (it stays NaN here)."""
    q = p if mask is None else len(list(mask))
    o = finalize_opts(mask, ddof, pca_on, want_vectors)
    flat = {"mean": np.zeros(q), "cov": np.zeros(q * q), "corr": np.zeros(q * q),
            "eigval": np.zeros(q), "eigvec": np.full(q * q, np.nan), "var_pct": np.zeros(q),
            "cum_pct": np.zeros(q)}
    pq = _i32(0)
    _check(_lib.stats_finalize(h, ctypes.byref(o), ctypes.byref(pq),
                               *(flat[k].ctypes.data for k in ("mean", "cov", "corr", "eigval",
                                                                "eigvec", "var_pct", "cum_pct"))))
    _release(h)
    qq = pq.value
    return {k: (v[:qq * qq].reshape(qq, qq) if k in ("cov", "corr", "eigvec") else v[:qq])
            for k, v in flat.items()}


def stats_finalize_groups(h: int, ngroups: int, p: int, mask=None, ddof: int = 1) -> dict:
    q = p if mask is None else len(list(mask))
    o = finalize_opts(mask, ddof)
    n = np.zeros(ngroups, dtype=np.int64)
    mean = np.zeros(ngroups * q)
    cov = np.zeros(ngroups * q * q)
    pq = _i32(0)
    _check(_lib.stats_finalize_groups(h, ctypes.byref(o), ctypes.byref(pq), n.ctypes.data,
                                      mean.ctypes.data, cov.ctypes.data))
    _release(h)
    qq = pq.value
    return {"n": n, "mean": mean[:ngroups * qq].reshape(ngroups, qq),
            "cov": cov[:ngroups * qq * qq].reshape(ngroups, qq, qq)}


def stats_serialize(h: int) -> bytes:
    n = ctypes.c_size_t(0)
    _check(_lib.stats_serialize(h, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(_lib.stats_serialize(h, buf, ctypes.byref(n)))
    _release(h)
    return buf.raw[:n.value]


def stats_deserialize(buf: bytes, cfg: Config) -> int:
    h = _vp()
    cbuf = ctypes.create_string_buffer(buf, len(buf))
    _check(_lib.stats_deserialize(cbuf, len(buf), ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def stats_kernel_time(h: int, which: int):
    n = _i64(0)
    ms = ctypes.c_double(0)
    _check(_lib.stats_kernel_time(h, which, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def stats_read_probe(bufs, nbytes, stream=None) -> float:
    """Milliseconds to read the given device buffers once (see stats.h)."""
    n = len(bufs)
    b = (ctypes.c_void_p * max(n, 1))(*[_ptr(x) for x in bufs])
    nb = (ctypes.c_int64 * max(n, 1))(*[int(x) for x in nbytes])
    ms = ctypes.c_double(0)
    _check(_lib.stats_read_probe(b, nb, n, stream or 0, ctypes.byref(ms)))
    return ms.value


def stats_close(h: int) -> None:
    _lib.stats_close(h)
    _release(h)


def library_path() -> str:
    return LIB_PATH


def exported_symbols():
    return [n for n in list(_sig) + ["stats_close", "stats_last_error"]]
