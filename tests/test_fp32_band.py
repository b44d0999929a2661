"""The float32 filter's error band, pinned on the CPU.

A C emulation of the filter's float32 decision (tests/fp32_band.c: float32
coordinates relative to float64 cell anchors, float32 differences, fused
multiply-add accumulation) is run over 10^8 random pairs per workload shape
(dimension, eps, cell extent M = eps / sqrt(d), coordinate range), nine in ten
within a few 1e-6 of eps.  For every pair the float32 value must lie within the
proof's bounds lo(D64) <= D32 <= hi(D64) around the defined float64 value, so no
pair is ever decided IN with D64 > E2 or OUT with D64 <= E2; the band [T_in, T_out]
must stay a few 1e-6 of E2 wide.  The bounds are the proof's, written out again
in the C file from its statement (the library evaluates them on the device).
"""

import ctypes
import math
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))

# (name, d, eps, coordinate range): the shapes of the benchmark workloads
SHAPES = [
    ("blobs2d", 2, 100.0, 1e4),
    ("spreader3d_1e6", 3, 200.0, 1e5),
    ("sweep3d_eps200", 3, 200.0, 1e6),
    ("sweep3d_eps400", 3, 400.0, 1e6),
    ("sweep3d_eps800", 3, 800.0, 1e6),
    ("sweep3d_eps1600", 3, 1600.0, 1e6),
    ("mixture5d_eps1.5", 5, 1.5, 100.0),
    ("mixture5d_eps2", 5, 2.0, 100.0),
    ("mixture5d_eps3", 5, 3.0, 100.0),
    ("mixture7d_eps1.5", 7, 1.5, 100.0),
    ("mixture7d_eps2", 7, 2.0, 100.0),
    ("mixture7d_eps3", 7, 3.0, 100.0),
    ("clouds2d_eps0.25", 2, 0.25, 100.0),
    ("clouds3d_eps0.5", 3, 0.5, 100.0),
    ("clouds5d_eps0.6", 5, 0.6, 100.0),
    ("d8_eps1", 8, 1.0, 100.0),
]
PAIRS = int(os.environ.get("BAND_PAIRS", 100_000_000))


@pytest.fixture(scope="module")
def band_lib(tmp_path_factory):
    out = tmp_path_factory.mktemp("band") / "fp32_band.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                    "-fPIC", "-shared", "-o", str(out), os.path.join(HERE, "fp32_band.c"), "-lm"],
                   check=True)
    lib = ctypes.CDLL(str(out))
    lib.band_check.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int64, ctypes.c_uint64, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_double)]
    lib.band_check.restype = None
    return lib


def _run(lib, d, eps, M, domain, pairs, seed, drop_eta=0):
    out = (ctypes.c_double * 9)()
    lib.band_check(d, eps, M, domain, pairs, seed, drop_eta, out)
    return list(out)


@pytest.mark.slow
@pytest.mark.parametrize("name,d,eps,domain", SHAPES, ids=[s[0] for s in SHAPES])
def test_band_bounds_hold(band_lib, name, d, eps, domain):
    M = eps / math.sqrt(d)
    hi, lo, wrong_in, wrong_out, band, mx_abs, tin, tout, inside = _run(
        band_lib, d, eps, M, domain, PAIRS, 1912062550 + d)
    assert hi <= 0.0, f"{name}: D32 above hi(D64) by {hi:.3e} E2"
    assert lo <= 0.0, f"{name}: D32 below lo(D64) by {-lo:.3e} E2"
    assert wrong_in == 0 and wrong_out == 0
    # the band is narrow (a few 1e-6 of E2) and the draws reach it on both sides
    assert 0.0 < tout - tin < 1e-5
    assert tin < 1.0 < tout
    assert band > 0 and 0.3 * PAIRS < inside < 0.7 * PAIRS
    # the bound is not vacuous: the largest error seen is a sizeable part of it
    assert mx_abs > 0.05 * (tout - tin)


def test_band_catches_a_dropped_error_term(band_lib):
    """A planted mistake (the coordinate error term eta left out of the bounds, as
    if the float32 coordinates were exact) must be caught by the same draws."""
    for d, eps, domain in ((3, 200.0, 1e6), (2, 100.0, 1e4)):
        M = eps / math.sqrt(d)
        hi, lo, wrong_in, wrong_out, *_ = _run(band_lib, d, eps, M, domain, 2_000_000, 11, 1)
        assert hi > 0.0 or lo > 0.0 or wrong_in > 0 or wrong_out > 0
