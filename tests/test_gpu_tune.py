"""Autotuner: the chosen options are valid, results stay exact under them, and the
table survives a save / load round trip."""

import numpy as np
import pytest

from oracle import dbscan_o1
from tests.gpu_helpers import gpu_dbscan, log
from workloads import gaussian_mixture, seed_spreader_3d

pytestmark = pytest.mark.gpu


@pytest.fixture
def clean_table(gpu_lib):
    from paper_1912_06255_amd import binding

    binding.tune_clear()
    yield binding
    binding.tune_clear()


@pytest.mark.parametrize("mode", ["fp64", "fp32_filter"])
def test_tune_then_exact(mode, clean_table):
    import torch

    binding = clean_table
    n = 40_000
    X = seed_spreader_3d(n, domain=1e5 * (n / 1e6) ** (1 / 3), seed=401)
    want = dbscan_o1(X, 200.0, 10)
    log(f"tune 3d {mode}")
    Xt = torch.from_numpy(X).cuda()
    out = (torch.empty(n, dtype=torch.uint8, device="cuda"), torch.empty(n, dtype=torch.int32, device="cuda"))
    res = binding.tune(Xt, 200.0, 10, mode=mode, out=out)
    assert res["bcp_rounds"] in (0, 1) and 0 <= res["unit_level"] <= 5
    assert 1 <= res["bcp_split"] <= 64 and 0 <= res["fine_bits"] <= 8
    assert res["subcell_min"] in (2048, 512, 0)
    assert res["mark_split"] in (1, 2, 4, 8) and res["dense_group"] in (4, 8, 16, 24)
    assert res["trials"] >= 4 and res["ms"] > 0 and res["ms"] <= res["ms_default"]
    assert res["size_class"] == int(np.floor(np.log2(n)))
    # the tuning runs leave the instance's exact result
    assert np.array_equal(out[0].cpu().numpy(), want[0]) and np.array_equal(out[1].cpu().numpy(), want[1])
    # later calls of the class use the tuned options
    got = gpu_dbscan(X, 200.0, 10, mode=mode, tag=f"after tune {mode}")
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_tune_high_dim_and_table_round_trip(clean_table, tmp_path):
    import torch

    binding = clean_table
    rng = np.random.Generator(np.random.PCG64(402))
    Y = gaussian_mixture(8000, 5, 10, 1.0, 12.0, 0.05, rng)
    log("tune 5d")
    res = binding.tune(torch.from_numpy(Y).cuda(), 2.0, 10, mode="fp64")
    want = dbscan_o1(Y, 2.0, 10)
    got = gpu_dbscan(Y, 2.0, 10, tag="after tune 5d")
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])

    path = tmp_path / "tune.txt"
    binding.tune_save(str(path))
    lines = path.read_text().splitlines()
    assert lines[0] == "dbscan-tune 4" and len(lines) == 2
    f = lines[1].split()
    assert [int(v) for v in f[:10]] == [5, 0, res["size_class"], res["bcp_rounds"], res["unit_level"],
                                        res["bcp_split"], res["fine_bits"], res["subcell_min"],
                                        res["mark_split"], res["dense_group"]]
    binding.tune_clear()
    binding.tune_save(str(path.with_suffix(".empty")))
    assert path.with_suffix(".empty").read_text().splitlines() == ["dbscan-tune 4"]
    binding.tune_load(str(path))
    binding.tune_save(str(path.with_suffix(".again")))
    assert path.with_suffix(".again").read_text().splitlines() == lines

    # older files load, the options they lack reading as automatic: version 1 has no
    # sub-cell threshold, versions 1 and 2 no MarkCore split or cell-by-cell threshold,
    # and up to version 3 the sub-cell threshold of d > 3 was unused
    old = tmp_path / "v1.txt"
    old.write_text("dbscan-tune 1\n3 1 13 0 1 2 0 1.5\n")
    binding.tune_clear()
    binding.tune_load(str(old))
    binding.tune_save(str(path.with_suffix(".v1")))
    assert path.with_suffix(".v1").read_text().splitlines() == ["dbscan-tune 4", "3 1 13 0 1 2 0 2048 4 8 1.5"]
    old2 = tmp_path / "v2.txt"
    old2.write_text("dbscan-tune 2\n2 0 12 1 1 2 0 512 0.5\n")
    binding.tune_clear()
    binding.tune_load(str(old2))
    binding.tune_save(str(path.with_suffix(".v2")))
    assert path.with_suffix(".v2").read_text().splitlines() == ["dbscan-tune 4", "2 0 12 1 1 2 0 512 4 8 0.5"]
    old3 = tmp_path / "v3.txt"
    old3.write_text("dbscan-tune 3\n5 0 13 1 1 2 0 2048 4 8 1.0\n3 0 13 0 1 2 0 512 2 16 0.4\n")
    binding.tune_clear()
    binding.tune_load(str(old3))
    binding.tune_save(str(path.with_suffix(".v3")))
    assert path.with_suffix(".v3").read_text().splitlines() == [
        "dbscan-tune 4", "5 0 13 1 1 2 0 0 4 8 1", "3 0 13 0 1 2 0 512 2 16 0.4"]
    binding.tune_clear()
    binding.tune_load(str(path))

    bad = tmp_path / "bad.txt"
    bad.write_text("dbscan-tune 2\n5 0 13 1 9 2 0 2048 1.0\n")  # unit level out of range
    with pytest.raises(binding.DbscanError) as e:
        binding.tune_load(str(bad))
    assert e.value.code == binding.EINVAL
    bad3 = tmp_path / "bad3.txt"
    bad3.write_text("dbscan-tune 3\n5 0 13 1 1 2 0 2048 3 8 1.0\n")  # MarkCore split not a power of two
    with pytest.raises(binding.DbscanError):
        binding.tune_load(str(bad3))
    binding.tune_save(str(path.with_suffix(".after_bad")))
    assert path.with_suffix(".after_bad").read_text().splitlines() == lines
    with pytest.raises(binding.DbscanError):
        binding.tune_load(str(tmp_path / "missing.txt"))
