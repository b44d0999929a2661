"""Full cluster membership (every cluster of each point) against the oracle."""

import numpy as np
import pytest

from oracle import membership as oracle_membership
from tests.gpu_helpers import log
from tests.pins import MEMBER_PINS
from workloads import blobs_2d, gaussian_mixture

pytestmark = pytest.mark.gpu

MODES = ["fp64", "fp32_filter"]


def gpu_members(X, eps, mp, mode="fp64"):
    import torch

    from paper_1912_06255_amd import binding

    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    if X.ndim == 1:
        X = X[:, None]
    log(f"membership n={X.shape[0]} d={X.shape[1]} eps={eps!r} minPts={mp} mode={mode}")
    binding.dbscan(torch.from_numpy(X).cuda(), eps, mp, mode=mode)
    off, ids = binding.membership()
    return off.cpu().numpy(), ids.cpu().numpy()


def _equal(got, want):
    return np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("pin", sorted(MEMBER_PINS))
def test_membership_pins_on_gpu(pin, mode, gpu_lib):
    fails = MEMBER_PINS[pin](lambda X, eps, mp: gpu_members(X, eps, mp, mode))
    assert not fails, "\n".join(fails)


@pytest.mark.parametrize("mode", MODES)
def test_membership_random(mode, gpu_lib):
    rng = np.random.Generator(np.random.PCG64(701))
    cases = [
        (blobs_2d(3000, seed=702), 100.0, 10),
        (blobs_2d(3000, seed=703), 160.0, 25),
        (gaussian_mixture(3000, 3, 8, 1.0, 10.0, 0.1, rng), 0.9, 12),
        (gaussian_mixture(2500, 5, 8, 1.0, 8.0, 0.1, rng), 1.8, 12),
        (rng.integers(0, 14, size=(2500, 2)).astype(np.float64), 1.0, 4),  # exact-eps pairs
    ]
    multi = 0
    for X, eps, mp in cases:
        want = oracle_membership(X, eps, mp)
        got = gpu_members(X, eps, mp, mode)
        multi += int((np.diff(want[0]) > 1).sum())
        assert _equal(got, want), f"d={X.shape[1]} eps={eps} minPts={mp}"
    assert multi > 0, "the cases must hold points in several clusters"


def test_membership_edge_cases_and_errors(gpu_lib):
    import torch

    from paper_1912_06255_amd import binding

    log("membership n=0")
    binding.dbscan(torch.zeros((0, 2), dtype=torch.float64, device="cuda"), 1.0, 3)
    off, ids = binding.membership()
    assert off.cpu().tolist() == [0] and ids.numel() == 0
    X = np.array([[0.0, 0.0], [5.0, 5.0]])
    assert _equal(gpu_members(X, 1.0, 1), oracle_membership(X, 1.0, 1))
    assert _equal(gpu_members(X, 1.0, 3), oracle_membership(X, 1.0, 3))  # all noise
    # a too small ids buffer is refused
    Y = blobs_2d(2000, seed=704)
    binding.dbscan(torch.from_numpy(Y).cuda(), 100.0, 10)
    with pytest.raises(binding.DbscanError) as e:
        binding.membership(ids_cap=1)
    assert e.value.code == binding.EINVAL
    # after a batch the single-call state is gone
    b = binding.Batch([torch.from_numpy(Y).cuda()], [[(100.0, 10)]])
    b.run()
    with pytest.raises(binding.DbscanError) as e:
        binding.membership()
    assert e.value.code == binding.EINVAL


def test_membership_full_size_properties(gpu_lib):
    """1M-point 3D workload: each point's smallest cluster is its label, core points
    have exactly one cluster, ids ascend and are distinct (properties of the exact
    output that hold at any size; the labels themselves are checked against the
    oracle's hash elsewhere)."""
    import torch

    from paper_1912_06255_amd import binding
    from workloads import config_workload

    X = config_workload(1)[0].X
    log("membership full size n=1e6")
    core, lab = binding.dbscan(torch.from_numpy(X).cuda(), 200.0, 10, mode="fp32_filter")
    off, ids = binding.membership()
    core, lab, off, ids = (t.cpu().numpy() for t in (core, lab, off, ids))
    cnt = np.diff(off)
    assert off[0] == 0 and np.all(cnt >= 0) and off[-1] == ids.size
    assert np.all(cnt[core != 0] == 1)
    first = np.where(cnt > 0, ids[np.minimum(off[:-1], max(ids.size - 1, 0))], -1)
    assert np.array_equal(first, lab)
    multi = np.flatnonzero(cnt > 1)
    for i in multi[:1000]:
        s = ids[off[i]:off[i + 1]]
        assert np.all(np.diff(s) > 0)
