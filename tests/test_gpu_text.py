"""Fused CSV ingest on the GPU: the parse is bit-exact against strtod/strtoll
(the oracle's parser), chunks split inside lines give the same statistics as
the binary path, and malformed fields are reported with their byte offset."""
import math
import struct

import numpy as np
import pytest

import datagen
import oracle
from helpers import TABLE1_INT, aos_config, check_raw_against_oracle, current_stream, lib, to_dev

pytestmark = pytest.mark.gpu


def _text_dev(b: bytes):
    import torch
    return torch.frombuffer(bytearray(b) + b"\0" * 16, dtype=torch.uint8).to("cuda:0")


def _cfg(L, p=10, int_cols=TABLE1_INT):
    return aos_config(p=p, int_cols=int_cols, stream=current_stream())


@pytest.mark.parametrize("n", [1, 2, 1000, 50_003])
def test_table1_csv_matches_oracle_and_binary(n):
    L = lib()
    txt = datagen.table1_csv(21, n)
    rows = oracle.parse_csv(txt, 10, TABLE1_INT)
    x = datagen.table1_aos(21, n)
    assert np.array_equal(rows.view(np.uint64), x.view(np.uint64))
    h = L.stats_open(_cfg(L))
    try:
        used = L.stats_accumulate_text(h, _text_dev(txt), len(txt), is_last=True)
        assert used == len(txt)
        raw = L.stats_raw(h, 10)
    finally:
        L.stats_close(h)
    st = oracle.sufficient_stats(oracle.columns_of(rows), TABLE1_INT)
    check_raw_against_oracle(raw, st, TABLE1_INT)
    assert raw["s_int"][0] == n * (n + 1) // 2


def test_chunks_split_inside_lines():
    L = lib()
    n = 30_000
    txt = datagen.table1_csv(22, n)
    rng = np.random.default_rng(0)
    cuts = sorted(set(int(c) for c in rng.integers(1, len(txt), size=6))) + [len(txt)]
    h = L.stats_open(_cfg(L))
    hb = L.stats_open(_cfg(L))
    try:
        carry = b""
        pos = 0
        for k, c in enumerate(cuts):
            chunk = carry + txt[pos:c]
            pos = c
            last = k == len(cuts) - 1
            used = L.stats_accumulate_text(h, _text_dev(chunk), len(chunk), is_last=last)
            carry = chunk[used:]
        assert carry == b""
        L.stats_accumulate(hb, [to_dev(datagen.table1_aos(22, n))], n)
        r1, r2 = L.stats_raw(h, 10), L.stats_raw(hb, 10)
    finally:
        L.stats_close(h)
        L.stats_close(hb)
    assert r1["n"] == r2["n"] == n
    assert r1["s_int"] == r2["s_int"] and r1["C_int"] == r2["C_int"]


def _fuzz_values(count):
    w = datagen.fuzz_words(99, 3 * count)
    vals = []
    for k in range(count):
        kind = k % 4
        if kind == 0:   # any finite double in the supported decimal range
            v = struct.unpack("<d", struct.pack("<Q", int(w[k])))[0]
            if not math.isfinite(v) or v == 0 or not (1e-40 < abs(v) < 1e55):
                v = (int(w[k]) % 10**12) / 7.0
        elif kind == 1:  # around Table-1 magnitudes
            v = (int(w[k]) % 2**53) / 2**53 * 20 - 10
        elif kind == 2:  # integers as floats
            v = float(int(w[k]) % 10**15) * (-1 if k % 3 == 0 else 1)
        else:            # tiny and huge exponents inside the range
            v = (1 + (int(w[k]) % 1000) / 1000) * 10.0 ** (int(w[k]) % 90 - 40)
        vals.append(v)
    return vals


@pytest.mark.parametrize("fmt", ["%.17g", "%.15g", "%.6e", "%.20f"])
def test_decimal_parse_bit_exact_vs_strtod(fmt):
    L = lib()
    vals = _fuzz_values(300)
    h = L.stats_open(_cfg(L, p=1, int_cols=[False]))
    bad = []
    try:
        for v in vals:
            s = (fmt % v).encode()
            ref = oracle.parse_csv(s + b"\n", 1, [False])[0, 0]
            L.stats_reset(h)
            L.stats_accumulate_text(h, _text_dev(s + b"\n"), len(s) + 1, is_last=True)
            got = L.stats_raw(h, 1)["s_f64"][0]
            ref = ref + 0.0  # a column sum of -0.0 is +0.0 (IEEE addition from +0)
            if struct.pack("<d", got) != struct.pack("<d", ref):
                bad.append((s, got, ref))
    finally:
        L.stats_close(h)
    assert not bad, bad[:5]


def test_short_lines_and_digit_runs():
    """Segments with more line starts than the workgroup's line table (lines
    of 4 to 7 bytes: each thread then walks its own slice), next to fields
    whose digit runs (leading zeros, signs, 1 to 17 digits, with and without
    point and exponent) start at every offset of the four-character steps.
    Integers against strtoll exactly, decimals through strtod."""
    L = lib()
    rng = np.random.default_rng(6)
    m = 60_000
    short = b"".join(b"%d,%d\n" % (a, b) for a, b in zip(rng.integers(0, 10, m), rng.integers(1, 100, m)))
    lines = []
    for _ in range(8000):
        nz = int(rng.integers(0, 6))
        a = rng.choice([b"", b"-", b"+"]) + b"0" * nz + str(int(rng.integers(0, 10 ** int(rng.integers(1, 7))))).encode()
        nd = int(rng.integers(1, 18))
        digits = str(int(rng.integers(10 ** (nd - 1), 10 ** nd))).encode()
        pt = int(rng.integers(0, nd + 1))
        b = b"0" * int(rng.integers(0, 3)) + digits[:pt] + (b"." + digits[pt:] if pt < nd else b"")
        if rng.random() < 0.2:
            b += b"e%d" % int(rng.integers(-20, 21))
        lines.append(a + b"," + b + b"\n")
    txt = short + b"".join(lines) + short[: short.index(b"\n", len(short) // 2) + 1]
    rows = oracle.parse_csv(txt, 2, [True, False])
    h = L.stats_open(_cfg(L, p=2, int_cols=[True, False]))
    try:
        used = L.stats_accumulate_text(h, _text_dev(txt), len(txt), is_last=True)
        assert used == len(txt)
        raw = L.stats_raw(h, 2)
    finally:
        L.stats_close(h)
    st = oracle.sufficient_stats(oracle.columns_of(rows), [True, False])
    check_raw_against_oracle(raw, st, [True, False])


@pytest.mark.parametrize("width", [1, 10, 18, 25, 40])
def test_line_lengths_set_the_segment_size(width):
    """The fused kernel's segment size follows the chunk's sampled mean line
    length (lines of 25 to 100 bytes on average here pick segments of 24, 28,
    32, 36 and 40 KiB): each size parses three zero-padded integer columns and
    one decimal column, over two chunks, to the oracle's statistics."""
    L = lib()
    rng = np.random.default_rng(width)
    n = 120_000
    a = rng.integers(-9, 10, n)
    b = rng.integers(0, 10 ** 4, n)
    c = rng.normal(0.0, 1e3, n)
    fmt_a = b"%0" + str(width).encode() + b"d"
    lines = [fmt_a % x + b"," + (b"%d" % y).rjust(width, b"0") + b"," + (b"%d" % (i + 1)) + b"," + (b"%.6f" % z)
             + b"\n" for i, (x, y, z) in enumerate(zip(a, b, c))]
    txt = b"".join(lines)
    int_cols = [True, True, True, False]
    rows = oracle.parse_csv(txt, 4, int_cols)
    h = L.stats_open(_cfg(L, p=4, int_cols=int_cols))
    try:
        d = _text_dev(txt)
        half = len(txt) // 2
        used = L.stats_accumulate_text(h, d.data_ptr(), half, is_last=False)
        used += L.stats_accumulate_text(h, d.data_ptr() + used, len(txt) - used, is_last=True)
        assert used == len(txt)
        raw = L.stats_raw(h, 4)
    finally:
        L.stats_close(h)
    st = oracle.sufficient_stats(oracle.columns_of(rows), int_cols)
    check_raw_against_oracle(raw, st, int_cols)


def test_parse_errors_report_offsets():
    L = lib()
    good = b"1,2,3\n"
    for txt, off in [(good + b"4,x,6\n", 8), (good + b"4,5\n", 8), (good + b"4,,6\n", 8),
                     (good * 3 + b"1.5,2,3\n", 18)]:
        h = L.stats_open(L.make_config([(L.STATS_I64, 0, 0, 0), (L.STATS_I64, 0, 8, 0),
                                        (L.STATS_I64, 0, 16, 0)], [24], stream=current_stream()))
        try:
            L.stats_accumulate_text(h, _text_dev(txt), len(txt), is_last=True)
            with pytest.raises(L.StatsError) as e:
                L.stats_sync(h)
            assert e.value.code == L.STATS_E_PARSE
            assert f"offset {off}" in e.value.msg, (txt, e.value.msg)
        finally:
            L.stats_close(h)


def test_unaligned_device_chunks():
    # chunks that start at arbitrary byte offsets of one device buffer
    L = lib()
    n = 20_000
    txt = datagen.table1_csv(23, n)
    d = _text_dev(txt)
    h = L.stats_open(_cfg(L))
    try:
        pos, step = 0, 77_777
        while pos < len(txt):
            m = min(step, len(txt) - pos)
            pos += L.stats_accumulate_text(h, d.data_ptr() + pos, m, is_last=(pos + m == len(txt)))
        raw = L.stats_raw(h, 10)
    finally:
        L.stats_close(h)
    st = oracle.sufficient_stats(oracle.columns_of(datagen.table1_aos(23, n)), TABLE1_INT)
    check_raw_against_oracle(raw, st, TABLE1_INT)


def test_incomplete_last_line_is_carried():
    L = lib()
    h = L.stats_open(_cfg(L, p=2, int_cols=[True, True]))
    try:
        used = L.stats_accumulate_text(h, _text_dev(b"1,2\n3,4\n5,"), 10, is_last=False)
        assert used == 8
        used = L.stats_accumulate_text(h, _text_dev(b"5,6"), 3, is_last=True)
        assert used == 3
        raw = L.stats_raw(h, 2)
    finally:
        L.stats_close(h)
    assert raw["n"] == 3 and raw["s_int"] == [9, 12]
    assert raw["C_int"][0][1] == 1 * 2 + 3 * 4 + 5 * 6
