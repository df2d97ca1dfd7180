"""CSV -> fixed-width binary file on the GPU, and its validation.

The paper converts its CSV dataset once into a fixed-width binary file and
then works from the binary form (section "Data Representation and Sufficient
Statistics"), after checking the result: file size, row count, column
layout and sample records against the text (section "Validation and
Infrastructure Testing").  ``csv_to_binary`` streams a CSV file through the
library's GPU parser (``stats_text_to_binary``) in chunks and appends the
rows to a binary file in the handle's one-plane layout; ``validate_binary``
performs the checks, reading the sample records' text lines on the host
with Python's own correctly rounded ``float`` / exact ``int`` (an
independent reading of the same bytes, not the GPU parser).
"""
from __future__ import annotations

import os
import struct

from . import (STATS_F64, STATS_I32, STATS_I64, STATS_MEM_DEVICE, make_config, stats_close, stats_open,
               stats_text_to_binary)

_FMT = {STATS_I32: "i", STATS_I64: "q", STATS_F64: "d"}


def csv_to_binary(csv_path: str, bin_path: str, cols, row_bytes: int, is_int, chunk_bytes: int = 1 << 30,
                  stream=None) -> dict:
    """Converts every line of csv_path into fixed-width records appended to
    bin_path (created or truncated).  cols: (dtype, byte_offset) of each of
    the p fields in a record of row_bytes bytes; is_int: integer columns.
    Returns {"rows", "text_bytes", "chunks"}."""
    import torch

    from . import STATS_COL_INTEGER
    ccols = [(dt, 0, off, STATS_COL_INTEGER if (is_int[c] and dt == STATS_F64) else 0)
             for c, (dt, off) in enumerate(cols)]
    h = stats_open(make_config(ccols, [row_bytes], stream=stream))
    dev = torch.device("cuda:0")
    text_dev = torch.empty(chunk_bytes + 16, dtype=torch.uint8, device=dev)
    max_rows = chunk_bytes // 2 + 1  # a line holds at least one byte and its '\n'
    out_dev = torch.empty(max_rows * row_bytes, dtype=torch.uint8, device=dev)
    rows = chunks = 0
    total = os.path.getsize(csv_path)
    try:
        with open(csv_path, "rb") as fin, open(bin_path, "wb") as fout:
            carry = b""
            pos = 0
            while True:
                want = chunk_bytes - len(carry)
                data = fin.read(want)
                pos += len(data)
                buf = carry + data
                last = pos >= total
                if not buf:
                    break
                if len(buf) > chunk_bytes:
                    raise ValueError("chunk larger than the device buffer")
                text_dev[:len(buf)].copy_(torch.frombuffer(bytearray(buf), dtype=torch.uint8))
                got, used = stats_text_to_binary(h, text_dev, len(buf), [out_dev], max_rows,
                                                 STATS_MEM_DEVICE, is_last=last)
                if used == 0 and not last:
                    raise ValueError(f"no complete line in a chunk of {len(buf)} bytes")
                fout.write(out_dev[:got * row_bytes].cpu().numpy().tobytes())
                rows += got
                chunks += 1
                carry = buf[used:]
                if last:
                    break
    finally:
        stats_close(h)
    return {"rows": rows, "text_bytes": total, "chunks": chunks}


def _line_offsets(csv_path: str, wanted: list[int]) -> dict[int, bytes]:
    """The text of the lines whose indices are in wanted (one pass)."""
    want = set(wanted)
    out = {}
    with open(csv_path, "rb") as f:
        for k, line in enumerate(f):
            if k in want:
                out[k] = line.rstrip(b"\n")
                if len(out) == len(want):
                    break
    return out


def validate_binary(csv_path: str, bin_path: str, cols, row_bytes: int, is_int, samples: int = 3) -> dict:
    """The paper's checks of a converted file: its size is a whole number of
    records, the record count equals the CSV line count, and the first,
    middle and last records (plus evenly spaced ones when samples > 3) hold
    exactly the values of their text lines.  Returns a report; "ok" is True
    when every check passes."""
    size = os.path.getsize(bin_path)
    with open(csv_path, "rb") as f:
        nlines = sum(chunk.count(b"\n") for chunk in iter(lambda: f.read(1 << 24), b""))
    with open(csv_path, "rb") as f:
        f.seek(max(0, os.path.getsize(csv_path) - 1))
        if os.path.getsize(csv_path) and f.read(1) != b"\n":
            nlines += 1  # a final line without '\n'
    rows = size // row_bytes
    report = {"bin_bytes": size, "row_bytes": row_bytes, "rows": rows, "csv_lines": nlines,
              "size_ok": size % row_bytes == 0, "rows_ok": rows == nlines, "mismatches": []}
    idx = sorted({0, rows // 2, rows - 1} | {rows * k // max(samples, 1) for k in range(samples)}) if rows else []
    idx = [i for i in idx if 0 <= i < rows]
    lines = _line_offsets(csv_path, idx)
    with open(bin_path, "rb") as fb:
        for i in idx:
            fb.seek(i * row_bytes)
            rec = fb.read(row_bytes)
            if i not in lines:
                report["mismatches"].append((i, "no such line"))
                continue
            fields = lines[i].split(b",")
            if len(fields) != len(cols):
                report["mismatches"].append((i, "field count"))
                continue
            for c, (dt, off) in enumerate(cols):
                fmt = "<" + _FMT[dt]
                got = struct.unpack_from(fmt, rec, off)[0]
                want = int(fields[c]) if is_int[c] else float(fields[c])
                if dt == STATS_F64:
                    same = struct.pack("<d", float(want)) == struct.pack("<d", got)
                else:
                    same = got == want
                if not same:
                    report["mismatches"].append((i, c))
    report["records_checked"] = idx
    report["layout_ok"] = not report["mismatches"]
    report["ok"] = report["size_ok"] and report["rows_ok"] and report["layout_ok"]
    return report
