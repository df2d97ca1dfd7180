"""The C ABI without a GPU: every declared entry point is exported, and
argument checks that need no device reject bad configurations."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stats.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(stats_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["stats_open", "stats_accumulate", "stats_merge", "stats_finalize", "stats_raw",
                 "stats_accumulate_text", "stats_open_groups", "stats_accumulate_segmented",
                 "stats_finalize_groups", "stats_serialize", "stats_deserialize", "stats_close",
                 "stats_last_error", "stats_sync", "stats_kernel_time", "stats_group_raw"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2604_23826_amd as L
    lib = ctypes.CDLL(L.library_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(L.exported_symbols()) == set(declared_functions())


def test_open_rejects_bad_configurations_without_a_device():
    import paper_2604_23826_amd as L
    bad = [
        L.make_config([], [8]),                                    # p = 0
        L.make_config([(9, 0, 0, 0)], [8]),                        # unknown dtype
        L.make_config([(L.STATS_F64, 1, 0, 0)], [8]),              # plane out of range
        L.make_config([(L.STATS_F64, 0, 4, 0)], [8]),              # element outside stride
        L.make_config([(L.STATS_F64, 0, 0, 0)], [8], block_rows=1000),  # not a multiple of 1024
        L.make_config([(L.STATS_F64, 0, 0, 64)], [8]),             # unknown flag
    ]
    for cfg in bad:
        with pytest.raises(L.StatsError) as e:
            L.stats_open(cfg)
        assert e.value.code == L.STATS_E_ARG
    L.stats_close(0)  # NULL-safe


def test_package_has_no_cpu_fallback():
    src = open(os.path.join(ROOT, "paper_2604_23826_amd", "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_2604_23826_amd", "csrc")):
        body = open(os.path.join(ROOT, "paper_2604_23826_amd", "csrc", f)).read()
        assert "oracle" not in body.lower(), f
