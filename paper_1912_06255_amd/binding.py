"""Thin ctypes binding of the HIP library (include/dbscan.h).

Only argument marshalling happens here: PyTorch provides device memory and the
stream, every step of the computation runs in the library's kernels.  If the
shared library is missing this module raises; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
import re
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DBSCAN_HIP_LIB") or os.path.join(HERE, "libdbscan_hip.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "dbscan.h")

OK = 0
EINVAL = -1
ENOMEM = -2
EHIP = -3
ENONFINITE = -4
EINTERNAL = -5
ETOOLARGE = -6

OPTIONS = {"bcp_rounds": 1, "unit_level": 2, "fine_bits": 3, "force_recheck": 4, "batch_graph": 5,
           "bcp_split": 6, "filter_max_d": 7, "subcell_min": 8, "sparse": 9, "group_clouds": 10,
           "mark_split": 11, "dense_group": 12, "cells": 13}

PLAIN_FP64 = 0
FP32_FILTER = 1
MODES = {"fp64": PLAIN_FP64, "plain": PLAIN_FP64, "fp32_filter": FP32_FILTER, "filter": FP32_FILTER}


class DbscanError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_points", ctypes.c_int64),
        ("n_cells", ctypes.c_int64),
        ("n_unsafe", ctypes.c_int64),
        ("n_core", ctypes.c_int64),
        ("bcp_calls", ctypes.c_int64),
        ("uf_links", ctypes.c_int64),
        ("fp64_rechecks", ctypes.c_int64),
        ("pair_tests", ctypes.c_int64),
        ("key_bits", ctypes.c_int32),
        ("key_shift", ctypes.c_int32),
        ("status", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("filter_tin", ctypes.c_float),
        ("filter_tout", ctypes.c_float),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Instance(ctypes.Structure):
    _fields_ = [
        ("points", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("d", ctypes.c_int32),
        ("n_settings", ctypes.c_int32),
        ("eps", ctypes.POINTER(ctypes.c_double)),
        ("min_pts", ctypes.POINTER(ctypes.c_int32)),
        ("core_flags", ctypes.c_void_p),
        ("cluster_id", ctypes.c_void_p),
    ]


class Tuned(ctypes.Structure):
    _fields_ = [
        ("bcp_rounds", ctypes.c_int32),
        ("unit_level", ctypes.c_int32),
        ("bcp_split", ctypes.c_int32),
        ("fine_bits", ctypes.c_int32),
        ("subcell_min", ctypes.c_int32),
        ("ms", ctypes.c_float),
        ("ms_default", ctypes.c_float),
        ("trials", ctypes.c_int32),
        ("size_class", ctypes.c_int32),
        ("mark_split", ctypes.c_int32),
        ("dense_group", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_lock = threading.Lock()
_ctx: dict[int, ctypes.c_void_p] = {}
_last_n: dict[int, int] = {}  # n of the last dbscan() call per device (sizes membership output)


def load():
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1912_06255_amd.build`"
        )
    # PyTorch first: its HIP runtime is then the one the library binds to.  Loaded
    # the other way round, the library would pull in a second HIP runtime whose
    # device state and streams are not PyTorch's.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.dbscan_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.dbscan_ctx_destroy.argtypes = [vp]
    lib.dbscan_reserve.argtypes = [vp, i64, i32]
    lib.dbscan.argtypes = [vp, vp, i64, i32, f64, i32, i32, vp, vp, vp]
    lib.dbscan_approx.argtypes = [vp, vp, i64, i32, f64, i32, f64, i32, vp, vp, vp]
    lib.dbscan_get_stats.argtypes = [vp, vp, ctypes.POINTER(Stats)]
    lib.dbscan_batch.argtypes = [vp, ctypes.POINTER(Instance), i32, i32, vp]
    lib.dbscan_set_option.argtypes = [vp, i32, i64]
    lib.dbscan_get_option.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.dbscan_set_profiling.argtypes = [vp, ctypes.c_int]
    lib.dbscan_phase_times.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_float), i32]
    lib.dbscan_phase_stats.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_float),
                                       ctypes.POINTER(i32), i32]
    lib.dbscan_phase_name.argtypes = [i32]
    lib.dbscan_phase_name.restype = ctypes.c_char_p
    lib.dbscan_tune.argtypes = [vp, vp, i64, i32, f64, i32, i32, vp, vp, vp, ctypes.POINTER(Tuned)]
    lib.dbscan_tune_save.argtypes = [vp, ctypes.c_char_p]
    lib.dbscan_tune_load.argtypes = [vp, ctypes.c_char_p]
    lib.dbscan_tune_clear.argtypes = [vp]
    lib.dbscan_membership.argtypes = [vp, vp, vp, i64, ctypes.POINTER(i64), vp]
    lib.dbscan_noalloc.argtypes = [vp, i64, i32, f64, i32, i32, vp, vp, vp, vp]
    lib.dbscan_strerror.argtypes = [ctypes.c_int]
    lib.dbscan_strerror.restype = ctypes.c_char_p
    for f in ("dbscan_ctx_create", "dbscan_ctx_destroy", "dbscan_reserve", "dbscan", "dbscan_get_stats",
              "dbscan_set_profiling", "dbscan_phase_times", "dbscan_phase_stats", "dbscan_set_option", "dbscan_get_option",
              "dbscan_batch", "dbscan_tune", "dbscan_tune_save", "dbscan_tune_load", "dbscan_tune_clear",
              "dbscan_membership", "dbscan_approx", "dbscan_noalloc"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def header_functions() -> list[str]:
    """Names of the functions declared in include/dbscan.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(dbscan\w*)\s*\(", text, flags=re.M)))


def strerror(code: int) -> str:
    try:
        return load().dbscan_strerror(code).decode()
    except Exception:  # pragma: no cover - only used in messages
        return "error"


def _check(rc: int, what: str) -> None:
    if rc != OK:
        raise DbscanError(rc, what)


def context(device: int = 0) -> ctypes.c_void_p:
    """The per-process context of a device (created on first use)."""
    with _lock:
        if device not in _ctx:
            h = ctypes.c_void_p()
            _check(load().dbscan_ctx_create(ctypes.byref(h), device), "dbscan_ctx_create")
            _ctx[device] = h
        return _ctx[device]


def reserve(n: int, d: int, device: int = 0) -> None:
    _check(load().dbscan_reserve(context(device), int(n), int(d)), "dbscan_reserve")


def _stream_handle(device, stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def dbscan(points, eps: float, min_pts: int, mode="fp64", out=None, stream=None, check: bool = True,
           rho: float | None = None):
    """Exact DBSCAN of ``points`` (float64 CUDA tensor [n, d]); with ``rho``,
    approximate DBSCAN (``dbscan_approx``: core points between eps and eps(1 + rho)
    apart may or may not share a cluster).

    Returns ``(core uint8[n], cluster_id int32[n])`` on the same device.  With
    ``check`` the stream is synchronised and device-detected errors raise
    ``DbscanError``; without it the call stays asynchronous.
    """
    import torch

    if not (isinstance(points, torch.Tensor) and points.is_cuda):
        raise TypeError("points must be a CUDA (HIP) tensor")
    if points.dtype != torch.float64 or points.dim() != 2:
        raise TypeError("points must be float64 of shape [n, d]")
    points = points.contiguous()
    n, d = points.shape
    dev = points.device.index if points.device.index is not None else torch.cuda.current_device()
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    if out is None:
        core = torch.empty(n, dtype=torch.uint8, device=points.device)
        label = torch.empty(n, dtype=torch.int32, device=points.device)
    else:
        core, label = out
    sh = _stream_handle(dev, stream)
    _last_n[dev] = n
    if rho is None:
        rc = load().dbscan(
            context(dev), ctypes.c_void_p(points.data_ptr()), n, d, float(eps), int(min_pts), m,
            ctypes.c_void_p(core.data_ptr()), ctypes.c_void_p(label.data_ptr()), sh,
        )
    else:
        rc = load().dbscan_approx(
            context(dev), ctypes.c_void_p(points.data_ptr()), n, d, float(eps), int(min_pts),
            float(rho), m, ctypes.c_void_p(core.data_ptr()), ctypes.c_void_p(label.data_ptr()), sh,
        )
    _check(rc, "dbscan" if rho is None else "dbscan_approx")
    if check and n > 0:
        stats(dev, stream, raise_on_error=True)
    return core, label


def dbscan_noalloc(points, eps: float, min_pts: int, mode="fp64", out=None, status=None,
                   stream=None):
    """dbscan() through the allocation-free entry point (fixed device scratch, no
    context): for inputs within its size limit.  ``out`` (core, labels) and
    ``status`` (int32 tensor of one element, receives the status bits) are CUDA
    tensors supplied by the caller or allocated here.  Asynchronous."""
    import torch

    if not (isinstance(points, torch.Tensor) and points.is_cuda and points.dtype == torch.float64
            and points.dim() == 2):
        raise TypeError("points must be a float64 CUDA tensor [n, d]")
    points = points.contiguous()
    n, d = points.shape
    dev = points.device.index if points.device.index is not None else torch.cuda.current_device()
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    if out is None:
        out = (torch.empty(n, dtype=torch.uint8, device=points.device),
               torch.empty(n, dtype=torch.int32, device=points.device))
    st = ctypes.c_void_p(status.data_ptr()) if status is not None else None
    with torch.cuda.device(dev):
        rc = load().dbscan_noalloc(
            ctypes.c_void_p(points.data_ptr()), n, d, float(eps), int(min_pts), m,
            ctypes.c_void_p(out[0].data_ptr()), ctypes.c_void_p(out[1].data_ptr()), st,
            _stream_handle(dev, stream))
    _check(rc, "dbscan_noalloc")
    return out


def tune(points, eps: float, min_pts: int, mode="fp64", out=None, stream=None) -> dict:
    """Autotune the options for ``points``' class (d, mode, size) and keep the
    choice in the context; returns the chosen options and timings.  Synchronises."""
    import torch

    if not (isinstance(points, torch.Tensor) and points.is_cuda and points.dtype == torch.float64
            and points.dim() == 2):
        raise TypeError("points must be a float64 CUDA tensor [n, d]")
    points = points.contiguous()
    n, d = points.shape
    dev = points.device.index if points.device.index is not None else torch.cuda.current_device()
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    if out is None:
        out = (torch.empty(n, dtype=torch.uint8, device=points.device),
               torch.empty(n, dtype=torch.int32, device=points.device))
    res = Tuned()
    rc = load().dbscan_tune(
        context(dev), ctypes.c_void_p(points.data_ptr()), n, d, float(eps), int(min_pts), m,
        ctypes.c_void_p(out[0].data_ptr()), ctypes.c_void_p(out[1].data_ptr()),
        _stream_handle(dev, stream), ctypes.byref(res),
    )
    _check(rc, "dbscan_tune")
    return res.as_dict()


def tune_save(path: str, device: int = 0) -> None:
    _check(load().dbscan_tune_save(context(device), os.fsencode(path)), "dbscan_tune_save")


def tune_load(path: str, device: int = 0) -> None:
    _check(load().dbscan_tune_load(context(device), os.fsencode(path)), "dbscan_tune_load")


def tune_clear(device: int = 0) -> None:
    _check(load().dbscan_tune_clear(context(device)), "dbscan_tune_clear")


def membership(device: int = 0, stream=None, ids_cap: int | None = None):
    """Full cluster membership of the last ``dbscan`` call: ``(offsets int64[n+1],
    ids int32[total])`` on the device, the ids of point i at
    ``ids[offsets[i]:offsets[i+1]]``, ascending.  ``ids_cap`` overrides the size of
    the ids buffer (for tests of the size check)."""
    import torch

    lib = load()
    dev = torch.device("cuda", device)
    n = _last_n.get(device, 0)
    offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
    total = ctypes.c_int64()
    sh = _stream_handle(device, stream)
    _check(lib.dbscan_membership(context(device), ctypes.c_void_p(offsets.data_ptr()), None, 0,
                                 ctypes.byref(total), sh), "dbscan_membership")
    cap = int(total.value) if ids_cap is None else int(ids_cap)
    ids = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    _check(lib.dbscan_membership(context(device), ctypes.c_void_p(offsets.data_ptr()),
                                 ctypes.c_void_p(ids.data_ptr()), cap, ctypes.byref(total), sh),
           "dbscan_membership")
    return offsets, ids[: int(total.value)]


def stats(device: int = 0, stream=None, raise_on_error: bool = False) -> dict:
    """Synchronise the stream and return the counters of the last call."""
    st = Stats()
    rc = load().dbscan_get_stats(context(device), _stream_handle(device, stream), ctypes.byref(st))
    if raise_on_error:
        _check(rc, "dbscan (device)")
    d = st.as_dict()
    d["rc"] = rc
    return d


def set_profiling(on: bool, device: int = 0) -> None:
    _check(load().dbscan_set_profiling(context(device), 1 if on else 0), "dbscan_set_profiling")


def phase_times(device: int = 0, stream=None) -> dict:
    """Per-phase milliseconds of the last call (profiling must be on), each summed
    over every occurrence of the phase in that call."""
    return {k: ms for k, (ms, _) in phase_stats(device, stream).items()}


def phase_stats(device: int = 0, stream=None) -> dict:
    """Per phase of the last call: (milliseconds summed over its occurrences,
    number of occurrences).  Profiling must be on."""
    lib = load()
    buf = (ctypes.c_float * 32)()
    occ = (ctypes.c_int32 * 32)()
    k = lib.dbscan_phase_stats(context(device), _stream_handle(device, stream), buf, occ, 32)
    if k < 0:
        raise DbscanError(k, "dbscan_phase_stats")
    return {lib.dbscan_phase_name(i).decode(): (float(buf[i]), int(occ[i])) for i in range(k)}


def set_option(name: str, value: int, device: int = 0) -> None:
    _check(load().dbscan_set_option(context(device), OPTIONS[name], int(value)), f"set_option {name}")


def get_option(name: str, device: int = 0) -> int:
    v = ctypes.c_int64()
    _check(load().dbscan_get_option(context(device), OPTIONS[name], ctypes.byref(v)), f"get_option {name}")
    return int(v.value)


class Batch:
    """A batch description for dbscan_batch: clouds (float64 CUDA tensors [n, d])
    with their (eps, minPts) settings.  Output tensors [n_settings, n] are
    allocated once; keeping the Batch object alive keeps every pointer stable, so
    repeated run() calls replay the captured graph."""

    def __init__(self, clouds, settings, mode="fp32_filter"):
        import torch

        if len(clouds) != len(settings):
            raise ValueError("one settings list per cloud")
        self.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        self.clouds = []
        self.core = []
        self.label = []
        self._keep = []
        arr = (Instance * len(clouds))()
        for i, (X, st) in enumerate(zip(clouds, settings)):
            if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float64 and X.dim() == 2):
                raise TypeError("each cloud must be a float64 CUDA tensor [n, d]")
            X = X.contiguous()
            n, d = X.shape
            eps = (ctypes.c_double * len(st))(*[float(e) for e, _ in st])
            mp = (ctypes.c_int32 * len(st))(*[int(m) for _, m in st])
            core = torch.empty((len(st), n), dtype=torch.uint8, device=X.device)
            lab = torch.empty((len(st), n), dtype=torch.int32, device=X.device)
            arr[i] = Instance(X.data_ptr(), n, d, len(st), eps, mp, core.data_ptr(), lab.data_ptr())
            self.clouds.append(X)
            self.core.append(core)
            self.label.append(lab)
            self._keep += [eps, mp]
        self._arr = arr
        self.device = self.clouds[0].device.index if self.clouds and self.clouds[0].device.index is not None else 0

    def run(self, stream=None, check: bool = True):
        rc = load().dbscan_batch(context(self.device), self._arr, len(self.clouds), self.mode,
                                 _stream_handle(self.device, stream))
        _check(rc, "dbscan_batch")
        if check:
            stats(self.device, stream, raise_on_error=True)
        return self.core, self.label

    @property
    def points(self) -> int:
        return int(sum(X.shape[0] * c.shape[0] for X, c in zip(self.clouds, self.core)))
