"""Seeded synthetic input generators (test and benchmark inputs only).

This module is shared by the CPU oracle, the tests and the benchmark.  It
produces inputs shaped like the paper's workloads and computes none of the
statistics:

* Table-1 rows (section "Background and Motivation", Table 1): identifier A,
  B ~ U{3..8}, C ~ U{1..10}, D ~ U{1..100} and the deterministic columns
  E, F, G, H, cotC, I (and J, K), as FP64 row-major records, as a planar
  int32 + FP64 layout, or as CSV text lines.
* 32-column rows: the 10 Table-1 columns then 22 i.i.d. U{0..100} integers.
* Log-uniform group sizes.
* Gaussian rows with a random correlation (see ``gauss``).

Random draws come from Philox4x32-10 keyed by the seed with the global row
index as counter, so any row range can be produced independently, on the host
(``libdatagen.so``, plain C) or in HBM (``libdatagen_dev.so``, HIP); both give
identical bytes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
HOST_LIB = os.path.join(HERE, "libdatagen.so")
DEV_LIB = os.path.join(HERE, "libdatagen_dev.so")

TABLE1_COLUMNS = ["A", "B", "C", "D", "E", "F", "G", "H", "cotC", "I", "J", "K"]
HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> None:
    """Compile the host generator with gcc and the device generator with hipcc."""
    cmds = [
        ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", HOST_LIB,
         os.path.join(HERE, "gen_host.c"), "-lm"],
        ["/opt/rocm/bin/hipcc", *HIP_FLAGS, "-o", DEV_LIB, os.path.join(HERE, "gen_dev.hip")],
    ]
    for c in cmds:
        if verbose:
            print(" ".join(c), flush=True)
        subprocess.run(c, check=True, cwd=HERE)


_host = None
_dev = None
_dev_tables_set = False

_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int32
_vp = ctypes.c_void_p


def host() -> ctypes.CDLL:
    global _host
    if _host is None:
        if not os.path.exists(HOST_LIB):
            build()
        lib = ctypes.CDLL(HOST_LIB)
        lib.dg_table1_tables.restype = ctypes.c_int
        lib.dg_table1_tables.argtypes = [_vp] * 8
        lib.dg_philox.argtypes = [_vp, _vp, _vp]
        lib.dg_table1_aos.argtypes = [_u64, _i64, _i64, _i64, _i32, _vp]
        lib.dg_table1_planar.argtypes = [_u64, _i64, _i64, _i64, _vp]
        lib.dg_groups_aos.argtypes = [_u64, _i64, _i64, _i64, _vp]
        lib.dg_group_sizes.argtypes = [_u64, _i32, ctypes.c_double, ctypes.c_double, _vp]
        lib.dg_table1_csv_size.restype = _i64
        lib.dg_table1_csv_size.argtypes = [_u64, _i64, _i64, _i64]
        lib.dg_table1_csv.restype = _i64
        lib.dg_table1_csv.argtypes = [_u64, _i64, _i64, _i64, _vp, _i64]
        lib.dg_fuzz_words.argtypes = [_u64, _i64, _vp]
        _host = lib
    return _host


def tables() -> dict:
    """Table-1 lookup tables built with the host libm, plus the number of the
    15 exact-integer E cases that came out wrong (0 expected)."""
    t = {"E": np.zeros((6, 10)), "F": np.zeros((6, 100)), "G": np.zeros(10),
         "H": np.zeros(100), "cot": np.zeros(10), "I": np.zeros(10), "J": np.zeros(100),
         "K": np.zeros((10, 100), dtype=np.int32)}
    bad = host().dg_table1_tables(*(t[k].ctypes.data for k in ("E", "F", "G", "H", "cot", "I", "J", "K")))
    t["bad_exact_E"] = int(bad)
    return t


def philox(ctr, key) -> list[int]:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    host().dg_philox(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return [int(x) for x in o]


def table1_aos(seed: int, n: int, row0: int = 0, a0: int | None = None, ncols: int = 10) -> np.ndarray:
    """n Table-1 rows as an (n, ncols) float64 array; identifier a0.. (default row0 + 1)."""
    out = np.empty((n, ncols), dtype=np.float64)
    if n:
        host().dg_table1_aos(seed, row0, row0 + 1 if a0 is None else a0, n, ncols, out.ctypes.data)
    return out


PLANAR_DTYPES = [np.int32] * 8 + [np.float64, np.int32]


def table1_planar(seed: int, n: int, row0: int = 0, a0: int | None = None) -> list[np.ndarray]:
    """Columns A B C D E F G H cotC I as separate planes (int32, cotC float64)."""
    planes = [np.empty(n, dtype=dt) for dt in PLANAR_DTYPES]
    if n:
        ptrs = (ctypes.c_void_p * 10)(*[p.ctypes.data for p in planes])
        host().dg_table1_planar(seed, row0, row0 + 1 if a0 is None else a0, n, ptrs)
    return planes


def table1_planar_threaded(seed: int, n: int, threads: int = 16) -> list[np.ndarray]:
    """table1_planar(seed, n) with the rows split over host threads (the C
    generator is counter-based, so the bytes do not depend on the split)."""
    planes = [np.empty(n, dtype=dt) for dt in PLANAR_DTYPES]
    if n == 0:
        return planes
    from concurrent.futures import ThreadPoolExecutor
    cuts = [n * k // threads for k in range(threads + 1)]

    def fill(k):
        a, b = cuts[k], cuts[k + 1]
        if b > a:
            ptrs = (ctypes.c_void_p * 10)(*[p.ctypes.data + a * p.itemsize for p in planes])
            host().dg_table1_planar(seed, a, a + 1, b - a, ptrs)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(fill, range(threads)))
    return planes


def groups_aos(seed: int, n: int, row0: int, a0: int) -> np.ndarray:
    """(n, 32) float64: 10 Table-1 columns (identifier a0..) + 22 U{0..100}."""
    out = np.empty((n, 32), dtype=np.float64)
    if n:
        host().dg_groups_aos(seed, row0, a0, n, out.ctypes.data)
    return out


def group_sizes(seed: int, ngroups: int, lo: float = 1e3, hi: float = 1e7) -> np.ndarray:
    out = np.empty(ngroups, dtype=np.int64)
    host().dg_group_sizes(seed, ngroups, lo, hi, out.ctypes.data)
    return out


def table1_csv(seed: int, n: int, row0: int = 0, a0: int | None = None) -> bytes:
    a = row0 + 1 if a0 is None else a0
    size = host().dg_table1_csv_size(seed, row0, a, n)
    buf = ctypes.create_string_buffer(max(int(size), 1))
    got = host().dg_table1_csv(seed, row0, a, n, buf, size)
    assert got == size
    return buf.raw[:size]


def table1_csv_into(seed: int, n: int, row0: int, a0: int, addr: int, cap: int) -> int:
    """Write CSV lines into host memory at addr (capacity cap); returns bytes or -1."""
    return int(host().dg_table1_csv(seed, row0, a0, n, addr, cap))


def fuzz_words(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    if n:
        host().dg_fuzz_words(seed, n, out.ctypes.data)
    return out


# ---- device generation (pointers are device addresses as Python ints) -------

def dev() -> ctypes.CDLL:
    global _dev, _dev_tables_set
    if _dev is None:
        if not os.path.exists(DEV_LIB):
            raise RuntimeError(f"{DEV_LIB} is not built; run datagen.build()")
        lib = ctypes.CDLL(DEV_LIB)
        lib.dgd_set_tables.argtypes = [_vp] * 8
        lib.dgd_table1_aos.argtypes = [_u64, _i64, _i64, _i64, _i32, _vp, _vp]
        lib.dgd_table1_planar.argtypes = [_u64, _i64, _i64, _i64, _vp, _vp]
        lib.dgd_groups_aos.argtypes = [_u64, _i64, _vp, _vp, _i32, _i64, _vp, _vp]
        _dev = lib
    if not _dev_tables_set:
        t = tables()
        rc = _dev.dgd_set_tables(*(np.ascontiguousarray(t[k]).ctypes.data
                                   for k in ("E", "F", "G", "H", "cot", "I", "J", "K")))
        if rc != 0:
            raise RuntimeError("dgd_set_tables failed")
        _dev_tables_set = True
    return _dev


def _chk(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"{what} failed")


def dev_table1_aos(seed: int, n: int, out_ptr: int, row0: int = 0, a0: int | None = None,
                   ncols: int = 10, stream: int = 0) -> None:
    _chk(dev().dgd_table1_aos(seed, row0, row0 + 1 if a0 is None else a0, n, ncols, out_ptr, stream),
         "dgd_table1_aos")


def dev_table1_planar(seed: int, n: int, plane_ptrs, row0: int = 0, a0: int | None = None,
                      stream: int = 0) -> None:
    ptrs = (ctypes.c_void_p * 10)(*plane_ptrs)
    _chk(dev().dgd_table1_planar(seed, row0, row0 + 1 if a0 is None else a0, n, ptrs, stream),
         "dgd_table1_planar")


def dev_groups_aos(seed: int, row0: int, off_ptr: int, a0_ptr: int, ngroups: int, n: int,
                   out_ptr: int, stream: int = 0) -> None:
    _chk(dev().dgd_groups_aos(seed, row0, off_ptr, a0_ptr, ngroups, n, out_ptr, stream),
         "dgd_groups_aos")
