"""CPU tests of bench.py's helpers: the counter summaries count only while they
were taken on the current kernel sources, and the per-bin relative error
skips the bins far below a multipole's scale."""
import os
import shutil

import numpy as np

import bench

SOURCES = ("bk_kernels.hpp", "bk_fft.hpp", "bk_tables.hpp", "bk_tables.cpp", "bk_api.hip")


def _fake_tree(tmp_path):
    csrc = tmp_path / "paper_2405_14513_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in SOURCES:
        shutil.copy(os.path.join(bench.ROOT, "paper_2405_14513_amd", "csrc", name), csrc / name)
    (tmp_path / "profiles").mkdir()
    return csrc


def test_traffic_is_read_only_for_the_current_kernel_sources(tmp_path, monkeypatch):
    csrc = _fake_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic(256) is None  # no summary
    h = bench.kernel_source_hash()
    (tmp_path / "profiles" / "k3_contract_traffic_ng256.txt").write_text(
        f"kernel: k3\nhbm_bytes_per_launch: 8.5e+10\nkernel_source_hash: {h}\n")
    (tmp_path / "profiles" / "k2_ring_traffic_ng256.txt").write_text(
        f"kernel: k2\nhbm_bytes_per_estimate: 3.2e+09\nkernel_source_hash: {h}\n")
    assert bench.read_traffic(256) == 8.5e10
    assert bench.read_k2_traffic(256) == 3.2e9
    # any edit of a kernel source, comments included, retires both summaries
    with open(csrc / "bk_tables.cpp", "a") as f:
        f.write("// edited\n")
    assert bench.kernel_source_hash() != h
    assert bench.read_traffic(256) is None
    assert bench.read_k2_traffic(256) is None


def test_committed_summaries_name_a_source_hash():
    for ng in (256, 512):
        for kind in ("k3_contract_traffic", "k2_ring_traffic"):
            txt = open(os.path.join(bench.ROOT, "profiles", f"{kind}_ng{ng}.txt")).read()
            assert "kernel_source_hash:" in txt and "command_fetch:" in txt and "command_write:" in txt


def test_per_bin_relative_skips_bins_below_the_floor():
    ref = np.array([[1.0, -2.0, 1e-6, np.nan], [4.0, 4.0, 4.0, 4.0]])
    B = np.array([[1.1, -2.0, 5.0, 7.0], [4.0, 4.4, 4.0, 3.0]])
    rel = bench.per_bin_relative(B, ref)
    assert np.isclose(rel[0], 0.1)  # the 1e-6 bin and the NaN bin are skipped
    assert np.isclose(rel[1], 0.25)
