"""CPU tests of the C ABI: the library loads, exports what the header declares,
and its host-side geometry matches the oracle bit for bit."""
import os
import re

import numpy as np
import pytest

from oracle.geometry import Binning, make_geometry
from paper_2405_14513_amd import bk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "bk.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bk_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = bk.lib()
    names = _declared()
    assert "bk_plan_create" in names and "bk_estimate" in names and len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize(
    "args",
    [
        (16, 3, 2.0, 5.0, 5, 3),
        (24, 2, 1.5, 8.0, 4, 3),
        (32, 4, 1.0, 32 / 3, 5, 5),
        (64, 20, 1.0, 64 / 3, 10, 10),
        (96, 20, 1.0, 32.0, 10, 10),
    ],
)
def test_host_triangle_counts_match_oracle_exactly(args):
    counts, ncomb = bk.bk_count_triangles(bk.make_binning(*args))
    g = make_geometry(Binning(*args))
    assert np.array_equal(counts, g.bin_counts().reshape(counts.shape))
    # the library folds each n -> -n partner into one canonical combination
    n = g.sides.plane[g.combos.sides]
    r = g.sides.ring[g.combos.sides]
    key = np.sort(r * 1000 + n, axis=1)
    key_mirror = np.sort(r * 1000 - n, axis=1)
    self_partner = np.all(key == key_mirror, axis=1)
    assert ncomb == self_partner.sum() + (~self_partner).sum() // 2


def test_host_errors():
    out = np.zeros(4, dtype=np.int64)
    import ctypes

    bad = bk.make_binning(16, 3, 2.0, 6.0, 5, 3)  # k1_max > N_g/3
    with pytest.raises(bk.BkError) as e:
        bk.bk_count_triangles(bad)
    assert e.value.status == bk.BK_ERR_ARG
    with pytest.raises(bk.BkError) as e:
        bk.bk_count_triangles(bk.make_binning(20, 3, 2.0, 5.0, 5, 3))  # 20 is not 2^a or 3*2^a
    assert e.value.status == bk.BK_ERR_ARG
    with pytest.raises(bk.BkError) as e:
        bk.bk_count_triangles(bk.make_binning(16, 3, 2.0, 5.0, 5, 3, l_max=14))
    assert e.value.status == bk.BK_ERR_ARG
    # every l up to 12 would be 91 outputs; a plan holds at most 64
    with pytest.raises(bk.BkError) as e:
        bk.bk_count_triangles(bk.make_binning(16, 3, 2.0, 5.0, 5, 3, l_max=12, m_max=12, even_l_only=0))
    assert e.value.status == bk.BK_ERR_ARG and "64" in bk.bk_last_error()
    with pytest.raises(bk.BkError) as e:
        bk.bk_count_triangles(bk.make_binning(16, 3, 2.0, 5.0, 5, 3, even_l_only=2))
    assert e.value.status == bk.BK_ERR_ARG
    # 9 x 10 / 2 = 45 outputs with every l <= 8 is accepted
    counts, n_comb = bk.bk_count_triangles(bk.make_binning(16, 3, 2.0, 5.0, 5, 3, l_max=8, m_max=8, even_l_only=0))
    assert n_comb > 0
    b = bk.make_binning(16, 3, 2.0, 5.0, 5, 3)
    st = bk.lib().bk_count_triangles(ctypes.byref(b), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 4, None)
    assert st == bk.BK_ERR_SIZE and "small" in bk.bk_last_error()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message, before touching a device."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _random_binnings(n, seed=2405):
    """Seeded binnings over small grids whose k1 edges often fall exactly on
    ring edges (integers and thirds), to exercise the interval tie rules."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        ng = int(rng.choice([8, 16, 24, 32, 48]))
        top = ng / 3.0
        grid = np.arange(1, int(3 * top) + 1) / 3.0  # multiples of 1/3 up to N_g/3
        k0, k1 = np.sort(rng.choice(grid, size=2, replace=False))
        if rng.random() < 0.3 and k0 < top:
            k1 = top
        out.append((ng, int(rng.integers(1, 6)), float(k0), float(k1), int(rng.integers(1, 9)),
                    int(rng.integers(1, 9))))
    return out


@pytest.mark.parametrize("args", _random_binnings(16))
def test_host_triangle_counts_match_oracle_on_random_binnings(args):
    counts, _ = bk.bk_count_triangles(bk.make_binning(*args))
    g = make_geometry(Binning(*args))
    assert np.array_equal(counts, g.bin_counts().reshape(counts.shape)), args
