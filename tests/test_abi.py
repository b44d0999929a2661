"""The C ABI library builds, loads and exports what include/dbscan.h declares.

Runs without a GPU: only symbol lookup and the pure-host functions are called.
"""

import ctypes
import os

import pytest

from paper_1912_06255_amd import binding


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_1912_06255_amd.build import build

        build()
    return binding.load()


def test_header_declares_the_entry_points():
    names = binding.header_functions()
    for f in ("dbscan", "dbscan_ctx_create", "dbscan_ctx_destroy", "dbscan_get_stats",
              "dbscan_reserve", "dbscan_strerror"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    for f in binding.header_functions():
        assert hasattr(lib, f), f"{f} declared in include/dbscan.h but not exported"


def test_strerror_covers_every_code(lib):
    seen = set()
    for code in (0, -1, -2, -3, -4, -5, -6):
        s = binding.strerror(code)
        assert s and s != "unknown error"
        seen.add(s)
    assert len(seen) == 7
    assert binding.strerror(-99) == "unknown error"


def test_null_arguments_are_rejected_without_touching_a_gpu(lib):
    assert lib.dbscan_ctx_create(None, 0) == binding.EINVAL
    assert lib.dbscan_ctx_destroy(None) == binding.EINVAL
    assert lib.dbscan_reserve(None, 10, 2) == binding.EINVAL
    st = binding.Stats()
    assert lib.dbscan_get_stats(None, None, ctypes.byref(st)) == binding.EINVAL
    # a NULL context is rejected before any argument or device is looked at
    assert lib.dbscan(None, None, 10, 2, 1.0, 3, 0, None, None, None) == binding.EINVAL
    assert lib.dbscan_approx(None, None, 10, 2, 1.0, 3, 0.01, 0, None, None, None) == binding.EINVAL


def test_stats_struct_matches_header():
    # int64 x8 + int32 x2 + uint32 x2 + float x2
    assert ctypes.sizeof(binding.Stats) == 8 * 8 + 4 * 4 + 4 * 2
    names = [f for f, _ in binding.Stats._fields_]
    assert names[-2:] == ["filter_tin", "filter_tout"]
