"""CSV -> fixed-width binary on the GPU (stats_text_to_binary) and rows
streamed from a binary file (stats_accumulate_file): the steps before and
around the single pass (sections "Data Representation and Sufficient
Statistics", "Validation and Infrastructure Testing", "System Overview").

The converted rows are compared bit for bit with the oracle's strtod /
strtoll parse of the same text and with the generator's binary rows; the
file-streamed statistics with the oracle on the same rows."""
import os

import numpy as np
import pytest

import datagen
import oracle
from helpers import TABLE1_INT, aos_config, check_raw_against_oracle, current_stream, lib, planar_config

pytestmark = pytest.mark.gpu


def _dev_bytes(b: bytes):
    import torch
    return torch.frombuffer(bytearray(b) + b"\0" * 16, dtype=torch.uint8).to("cuda:0")


def _empty(nbytes):
    import torch
    return torch.zeros(max(nbytes, 16), dtype=torch.uint8, device="cuda:0")


@pytest.mark.parametrize("n", [1, 3, 1000, 70_001])
def test_csv_to_fp64_rows_bit_exact(n):
    """80-byte FP64 records (integer columns as exact FP64 integers)."""
    L = lib()
    txt = datagen.table1_csv(31, n)
    ref = oracle.parse_csv(txt, 10, TABLE1_INT)
    h = L.stats_open(aos_config(stream=current_stream()))
    try:
        out = _empty(80 * n)
        rows, used = L.stats_text_to_binary(h, _dev_bytes(txt), len(txt), [out], n, is_last=True)
    finally:
        L.stats_close(h)
    assert rows == n and used == len(txt)
    got = out[:80 * n].cpu().numpy().view(np.float64).reshape(n, 10)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    assert np.array_equal(got.view(np.uint64), datagen.table1_aos(31, n).view(np.uint64))


@pytest.mark.parametrize("chunk", [4096, 1 << 16, 1 << 20])
def test_csv_to_int32_planes_in_chunks(chunk):
    """Nine int32 planes + one FP64 plane, the text cut into chunks inside
    lines (the caller passes the unconsumed tail again)."""
    import torch
    L = lib()
    n = 60_013
    txt = datagen.table1_csv(32, n)
    ref = datagen.table1_planar(32, n)
    h = L.stats_open(planar_config(stream=current_stream()))
    dts = [torch.int32] * 8 + [torch.float64, torch.int32]
    try:
        pos = row = 0
        planes = [torch.zeros(n, dtype=dt, device="cuda:0") for dt in dts]
        while pos < len(txt):
            piece = txt[pos:pos + chunk]
            last = pos + len(piece) == len(txt)
            views = [pl[row:] for pl in planes]
            got, used = L.stats_text_to_binary(h, _dev_bytes(piece), len(piece), views, n - row, is_last=last)
            assert used > 0
            pos += used
            row += got
    finally:
        L.stats_close(h)
    assert row == n
    for pl, r in zip(planes, ref):
        a = pl.cpu().numpy()
        assert a.dtype == r.dtype and np.array_equal(a.view(np.uint8), r.view(np.uint8))


def test_csv_short_lines_take_the_slice_walk():
    """More than 4096 line starts in a 32 KiB segment (lines of 4 bytes):
    the workgroup numbers its lines by slice counts instead of the table."""
    L = lib()
    n = 50_000
    vals = np.random.default_rng(3).integers(0, 100, size=n)
    txt = "".join(f"{v}\n" for v in vals).encode()
    cols = [(L.STATS_I64, 0, 0, 0)]
    h = L.stats_open(L.make_config(cols, [8], stream=current_stream()))
    try:
        out = _empty(8 * n)
        rows, used = L.stats_text_to_binary(h, _dev_bytes(txt), len(txt), [out], n, is_last=True)
    finally:
        L.stats_close(h)
    assert rows == n
    assert np.array_equal(out[:8 * n].cpu().numpy().view(np.int64), vals)


def test_csv_conversion_errors():
    L = lib()
    txt = b"1,2\n3,4\n5,x\n"
    cols = [(L.STATS_I32, 0, 0, 0), (L.STATS_I32, 0, 4, 0)]
    h = L.stats_open(L.make_config(cols, [8], stream=current_stream()))
    try:
        out = _empty(64)
        with pytest.raises(L.StatsError) as e:
            L.stats_text_to_binary(h, _dev_bytes(txt), len(txt), [out], 3, is_last=True)
        assert e.value.code == L.STATS_E_PARSE and "offset 8" in str(e.value)
        with pytest.raises(L.StatsError) as e:  # more lines than output rows
            L.stats_text_to_binary(h, _dev_bytes(b"1,2\n3,4\n"), 8, [out], 1, is_last=True)
        assert e.value.code == L.STATS_E_ARG
        with pytest.raises(L.StatsError) as e:  # beyond int32
            L.stats_text_to_binary(h, _dev_bytes(b"1,2147483648\n"), 13, [out], 1, is_last=True)
        assert e.value.code == L.STATS_E_PARSE
        rows, used = L.stats_text_to_binary(h, _dev_bytes(b"-2147483648,2147483647\n"), 23, [out], 1,
                                            is_last=True)
        assert rows == 1 and list(out[:8].cpu().numpy().view(np.int32)) == [-2147483648, 2147483647]
    finally:
        L.stats_close(h)
    # FP32 output is refused (a decimal rounded twice)
    h = L.stats_open(L.make_config([(L.STATS_F32, 0, 0, 0)], [4], stream=current_stream()))
    try:
        with pytest.raises(L.StatsError) as e:
            L.stats_text_to_binary(h, _dev_bytes(b"1.5\n"), 4, [_empty(16)], 1, is_last=True)
        assert e.value.code == L.STATS_E_ARG
    finally:
        L.stats_close(h)


def test_csv_file_to_binary_file_and_validation(tmp_path):
    """The whole conversion tool: a CSV file through the GPU in chunks to an
    80-byte-record file, then the paper's checks (size, row count, first /
    middle / last records re-read from the text on the host)."""
    from paper_2604_23826_amd import convert
    L = lib()
    n = 123_457
    txt = datagen.table1_csv(33, n)
    csv = tmp_path / "t.csv"
    csv.write_bytes(txt)
    binp = tmp_path / "t.bin"
    cols = [(L.STATS_F64, 8 * c) for c in range(10)]
    info = convert.csv_to_binary(str(csv), str(binp), cols, 80, TABLE1_INT, chunk_bytes=1 << 20,
                                 stream=current_stream())
    assert info["rows"] == n and info["chunks"] > 1
    rep = convert.validate_binary(str(csv), str(binp), cols, 80, TABLE1_INT, samples=7)
    assert rep["ok"], rep
    x = np.fromfile(binp, dtype=np.float64).reshape(n, 10)
    assert np.array_equal(x.view(np.uint64), datagen.table1_aos(33, n).view(np.uint64))
    # a damaged record is caught by the sample check
    with open(binp, "r+b") as f:
        f.seek(80 * (n // 2) + 8 * 3)
        f.write(np.float64(-1.0).tobytes())
    rep = convert.validate_binary(str(csv), str(binp), cols, 80, TABLE1_INT)
    assert not rep["ok"] and rep["mismatches"] == [(n // 2, 3)]


@pytest.mark.parametrize("n,staging", [(1, 0), (250_001, 65_536), (1_000_000, 0)])
def test_rows_streamed_from_a_file(tmp_path, n, staging):
    """80-byte Table-1 records read from a file (positioned reads into the
    pinned ring) give the oracle's statistics; offset and partial reads."""
    L = lib()
    x = datagen.table1_aos(34, n + 7)
    path = tmp_path / "rows.bin"
    head = b"HEADER!!" * 3  # 24 bytes before the first record
    path.write_bytes(head + x.tobytes())
    h = L.stats_open(aos_config(stream=current_stream(), staging_rows=staging))
    try:
        L.stats_accumulate_file(h, str(path), len(head) + 80 * 7, n)
        raw = L.stats_raw(h, 10)
    finally:
        L.stats_close(h)
    rows = x[7:]
    st = oracle.sufficient_stats(oracle.columns_of(rows), TABLE1_INT)
    check_raw_against_oracle(raw, st, TABLE1_INT)


def test_file_errors(tmp_path):
    L = lib()
    path = tmp_path / "short.bin"
    path.write_bytes(b"\0" * (80 * 10))
    h = L.stats_open(aos_config(stream=current_stream()))
    try:
        with pytest.raises(L.StatsError) as e:
            L.stats_accumulate_file(h, str(tmp_path / "missing.bin"), 0, 1)
        assert e.value.code == L.STATS_E_IO
        with pytest.raises(L.StatsError) as e:
            L.stats_accumulate_file(h, str(path), 80, 10)  # one record short
        assert e.value.code == L.STATS_E_IO
        L.stats_accumulate_file(h, str(path), 0, 10)
        assert L.stats_raw(h, 10)["n"] == 10
    finally:
        L.stats_close(h)
    h = L.stats_open(planar_config(stream=current_stream()))
    try:
        with pytest.raises(L.StatsError) as e:
            L.stats_accumulate_file(h, str(path), 0, 1)
        assert e.value.code == L.STATS_E_ARG
    finally:
        L.stats_close(h)


def test_decimal_range_boundary():
    """The exact-ratio conversion takes decimal fields w * 10^q (w the
    written significand, q the exponent of its last digit) below 10^73 in
    magnitude with q >= -57: the values just inside parse to the correctly
    rounded double; just outside (1e74, a last digit at 10^-58) the field is
    refused with STATS_E_PARSE and the line's offset, never rounded wrongly."""
    import struct
    L = lib()
    cols = [(L.STATS_F64, 0, 0, 0), (L.STATS_F64, 0, 8, 0)]
    inside = [b"1e73", b"-9.999999999999999e72", b"1e-57", b"-1.5e-56", b"123456789012345678901e52",
              b"0.000000000000000000000000000000000000000000000000000000001"]
    outside = [b"1e74", b"9e73", b"1e-58", b"1.0e-57", b"1e100", b"-1e-300"]
    h = L.stats_open(L.make_config(cols, [16], stream=current_stream()))
    try:
        txt = b"".join(v + b",1\n" for v in inside)
        out = _empty(16 * len(inside))
        rows, used = L.stats_text_to_binary(h, _dev_bytes(txt), len(txt), [out], len(inside), is_last=True)
        assert rows == len(inside) and used == len(txt)
        got = out[:16 * len(inside)].cpu().numpy().view(np.float64).reshape(-1, 2)[:, 0]
        for g, v in zip(got, inside):
            ref = float(v.decode())
            assert struct.pack("<d", g) == struct.pack("<d", ref), (v, g, ref)
    finally:
        L.stats_close(h)
    for v in outside:
        # a fresh handle each: offsets count from the start of a handle's text
        h = L.stats_open(L.make_config(cols, [16], stream=current_stream()))
        try:
            line = b"2,3\n" + v + b",1\n"
            with pytest.raises(L.StatsError) as e:
                L.stats_text_to_binary(h, _dev_bytes(line), len(line), [_empty(32)], 2, is_last=True)
            assert e.value.code == L.STATS_E_PARSE and "offset 4" in str(e.value), v
        finally:
            L.stats_close(h)
