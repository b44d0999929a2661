"""Full-size workloads through dbscan_batch in the benchmark's launch configuration
(one batch per workload, float32 filter mode, the captured graph replayed) against
the oracle's hashes of core flags and cluster ids.

The hashes in tests/golden/full_size_hashes.json come from
tests/golden/make_full_size_hashes.py, which runs only the C oracle (itself pinned
to the brute-force oracle) on the seeded generators.  Covered bit for bit: the 2D
blobs, the 1M-point 3D cloud, both 2M-point mixtures (5D and 7D) at eps 1.5, 2 and
3 (also with the float32 filter taking every decision, the precision form), every
one of the 256 clouds, and the 10M-point sweep at all 16 of its settings (eps 200,
400, 800 and 1600, four minPts each; the oracle took about 16 minutes per setting at
eps 1600).  test_gpu_full_size.py adds sampled checks of the same runs.
"""

import numpy as np
import pytest

from tests.gpu_helpers import digest, full_size_cases, log
from workloads import config_workload

pytestmark = pytest.mark.gpu


def _name(prefix, eps, mp):
    return f"{prefix}_eps{eps:g}_mp{mp}"


def _run_batch(clouds, settings, mode="fp32_filter"):
    import torch

    from paper_1912_06255_amd import binding

    dev = [torch.from_numpy(X).cuda() for X in clouds]
    b = binding.Batch(dev, settings, mode=mode)
    b.run()  # capture and first replay
    for c, l in zip(b.core, b.label):
        c.fill_(7)
        l.fill_(-7)
    b.run()  # a replay writes every output again
    out = [(c.cpu().numpy(), l.cpu().numpy()) for c, l in zip(b.core, b.label)]
    st = binding.stats(raise_on_error=True)
    del b, dev
    torch.cuda.empty_cache()
    return out, st


def test_sweep_batch_matches_oracle_hashes(gpu_lib):
    cases = full_size_cases()
    I = config_workload(3)[0]
    settings = list(zip(I.eps, I.min_pts))
    log(f"sweep batch n={I.n} settings={len(settings)}")
    ((core, lab),), _ = _run_batch([I.X], [settings])
    for s, (eps, mp) in enumerate(settings):
        name = _name("sweep3d_n10000000", eps, mp)
        assert name in cases, f"{name} has no oracle hash"
        assert digest(core[s], lab[s]) == cases[name]["sha256"], name
        assert int(core[s].sum()) == cases[name]["n_core"], name


def test_multicloud_batch_matches_oracle_hashes(gpu_lib):
    rec = full_size_cases()["multicloud_256"]
    inst = config_workload(4)
    assert len(inst) == len(rec["clouds"]) == 256
    log(f"multi-cloud batch clouds={len(inst)} points={sum(I.n for I in inst)}")
    out, _ = _run_batch([I.X for I in inst], [list(zip(I.eps, I.min_pts)) for I in inst])
    bad = []
    for ci, (I, want, (core, lab)) in enumerate(zip(inst, rec["clouds"], out)):
        assert (I.n, I.d, I.eps[0], I.min_pts[0]) == (want["n"], want["d"], want["eps"], want["min_pts"])
        if digest(core[0], lab[0]) != want["sha256"]:
            bad.append(f"cloud {ci} (n={I.n}, d={I.d})")
    assert not bad, bad[:20]


@pytest.mark.parametrize("filter_max_d", [-1, 8])
@pytest.mark.parametrize("which", [0, 1])
def test_mixture_batch_matches_oracle_hashes(which, filter_max_d, gpu_lib):
    """The 5D / 7D mixtures at their three eps; with filter_max_d = 8 the float32
    filter takes the pair decisions in these dimensions too (the precision form),
    with its float64 rechecks counted."""
    from paper_1912_06255_amd import binding

    cases = full_size_cases()
    I = config_workload(2)[which]
    settings = list(zip(I.eps, I.min_pts))
    binding.set_option("filter_max_d", filter_max_d)
    try:
        log(f"mixture d={I.d} batch filter_max_d={filter_max_d}")
        ((core, lab),), st = _run_batch([I.X], [settings])
    finally:
        binding.set_option("filter_max_d", -1)
    for s, (eps, mp) in enumerate(settings):
        name = _name(f"mixture{I.d}d_n2000000", eps, mp)
        assert digest(core[s], lab[s]) == cases[name]["sha256"], name
    if filter_max_d == 8:
        assert st["fp64_rechecks"] > 0  # the band is reached, and those pairs re-decided
