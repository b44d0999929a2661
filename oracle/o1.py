"""ctypes front end of the C oracle O1 (test infrastructure only).

``build_o1()`` compiles ``o1.c`` with gcc into ``_o1.so`` next to it, with
-ffp-contract=off so that the float64 decisions are the defined ones.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "o1.c")
_LIB = os.path.join(_HERE, "_o1.so")
_lib = None

ERRORS = {-1: "invalid argument", -2: "out of memory", -4: "bucket range", -5: "non-finite input"}


def build_o1(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        cmd = [
            "gcc", "-O3", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm",
        ]
        subprocess.run(cmd, check=True)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_o1(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.o1_dbscan.restype = ctypes.c_int
        lib.o1_dbscan.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
        ]
        lib.o1_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def o1_available() -> bool:
    try:
        _load()
        return True
    except OSError:
        return False


def o1_threads() -> int:
    return int(_load().o1_max_threads())


def dbscan_o1(X, eps: float, min_pts: int, threads: int = 0):
    """Exact DBSCAN (same contract as ``dbscan_brute``) through the C oracle."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    if X.ndim == 1:
        X = X[:, None]
    n, d = X.shape
    core = np.zeros(n, dtype=np.uint8)
    label = np.zeros(n, dtype=np.int32)
    rc = _load().o1_dbscan(
        X.ctypes.data, n, d, float(eps), int(min_pts), int(threads),
        core.ctypes.data, label.ctypes.data,
    )
    if rc != 0:
        raise ValueError(f"o1_dbscan failed: {ERRORS.get(rc, rc)}")
    return core, label
