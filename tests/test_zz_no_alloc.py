"""The allocation-free entry point dbscan_noalloc (scratch in a fixed device array).

CPU part: the size limit is refused before any device work.  GPU part: two calls
in a row (the second smaller, so the array holds the first call's leftovers)
through the C ABI, each against dbscan() on the same input, in both modes; an
empty call writes a zero status.
"""

import ctypes

import numpy as np
import pytest

from paper_1912_06255_amd import binding
from tests.gpu_helpers import log
from workloads import blobs_2d, seed_spreader_3d


def _fn():
    f = binding.load().dbscan_noalloc
    return f


def test_noalloc_size_limit_refused_on_host():
    f = _fn()
    # refused before any HIP call (so this runs without a GPU)
    assert f(1, 348_993, 3, 1.0, 5, 0, 1, 1, None, None) == binding.ETOOLARGE
    assert f(1, 177_433, 8, 1.0, 5, 0, 1, 1, None, None) == binding.ETOOLARGE
    assert f(None, 100, 3, 1.0, 5, 0, None, None, None, None) == binding.EINVAL
    assert f(1, 100, 9, 1.0, 5, 0, 1, 1, None, None) == binding.EINVAL
    assert f(1, 100, 3, 1.0, 5, 7, 1, 1, None, None) == binding.EINVAL
    assert binding.strerror(binding.ETOOLARGE) != "unknown error"


def _noalloc(X, eps, mp, mode):
    import torch

    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    n, d = Xd.shape
    core = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    lab = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    log(f"dbscan_noalloc n={n} d={d} eps={eps} minPts={mp} mode={mode}")
    rc = _fn()(ctypes.c_void_p(Xd.data_ptr()), n, d, float(eps), int(mp), binding.MODES[mode],
               ctypes.c_void_p(core.data_ptr()), ctypes.c_void_p(lab.data_ptr()),
               ctypes.c_void_p(status.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    assert rc == binding.OK, binding.strerror(rc)
    torch.cuda.synchronize()
    return core.cpu().numpy(), lab.cpu().numpy(), int(status.cpu().item())


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["fp64", "fp32_filter"])
def test_noalloc_matches_dbscan_two_calls(mode, gpu_lib):
    import torch

    A = seed_spreader_3d(300_000, domain=1e5 * 0.3 ** (1.0 / 3.0), seed=77)
    B = blobs_2d(40_000, seed=78)
    for X, eps, mp in ((A, 200.0, 10), (B, 100.0, 10)):
        core, lab, status = _noalloc(X, eps, mp, mode)
        want = gpu_lib.dbscan(torch.from_numpy(X).cuda(), eps, mp, mode=mode)
        assert status == 0
        assert np.array_equal(core, want[0].cpu().numpy())
        assert np.array_equal(lab, want[1].cpu().numpy())
        assert core.sum() > 0 and lab.max() >= 0


@pytest.mark.gpu
def test_noalloc_empty_and_nonfinite(gpu_lib):
    import torch

    core, lab, status = _noalloc(np.zeros((0, 2)), 1.0, 5, "fp64")
    assert status == 0 and core.size == 0
    X = blobs_2d(2_000, seed=5)
    X[17, 1] = np.nan
    core, lab, status = _noalloc(X, 100.0, 10, "fp64")
    assert status & 1  # DBSCAN_STATUS_NONFINITE
    # and the next call is clean again
    core, lab, status = _noalloc(blobs_2d(2_000, seed=6), 100.0, 10, "fp32_filter")
    want = gpu_lib.dbscan(torch.from_numpy(blobs_2d(2_000, seed=6)).cuda(), 100.0, 10)
    assert status == 0 and np.array_equal(lab, want[1].cpu().numpy())
