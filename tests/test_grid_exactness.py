"""The reduced-grid evaluation of the triple products (Eq. 8), pinned on the CPU.

The library sums each combination on an m x m grid instead of N_g x N_g.
With every mode of ring r inside |u_x|, |u_y| <= U_r, the only solutions of
u_1 + u_2 + u_3 = 0 (mod m) are the closed triangles once m > U_1 + U_2 + U_3,
so S on the m-grid is (m / N_g)^2 times S on the full grid.  These tests check
that claim with numpy FFTs against the oracle's full-grid triple sums, and
check that one grid point fewer does alias, so the bound is the one in use.
"""
import numpy as np

from oracle.estimator import fourier_field, triple_sums_fft
from oracle.geometry import Binning, make_geometry
from synth import FieldRecipe, make_field


def _D_on_grid(Delta, modes, plane, m):
    ng = Delta.shape[0]
    folded = np.zeros((m, m), dtype=np.complex128)
    np.add.at(folded, (modes[:, 0] % m, modes[:, 1] % m), Delta[modes[:, 0] % ng, modes[:, 1] % ng, plane % ng])
    return np.fft.fft2(folded)


def _setup(ng=32, seed=5):
    b = Binning(ng, 4, 1.0, ng / 3, 5, 4)
    g = make_geometry(b)
    delta = make_field(FieldRecipe(ng, n_s=-2.0, f_ng=0.5, beta=0.5, seed=seed))
    Delta = fourier_field(delta, b.box_len)
    U = [int(np.abs(mo).max()) for mo in g.rings.modes]  # |u_x| and |u_y| share the bound
    return b, g, Delta, U


def _S_on_grid(b, g, Delta, rows, m_of_row):
    ng = b.ng
    out = np.empty(len(rows), dtype=np.complex128)
    for k, (row, m) in enumerate(zip(rows, m_of_row)):
        prod = np.ones((m, m), dtype=np.complex128)
        for s in g.combos.sides[row]:
            r, n = int(g.sides.ring[s]), int(g.sides.plane[s])
            prod *= _D_on_grid(Delta, g.rings.modes[r - 1], n, m)
        out[k] = prod.sum() * (ng / m) ** 2 / (b.volume * ng * ng)
    return out


def test_reduced_grid_sum_equals_full_grid_sum():
    b, g, Delta, U = _setup()
    rng = np.random.default_rng(0)
    rows = rng.choice(len(g.combos.ntri), size=60, replace=False)
    full = triple_sums_fft(g, Delta, rows)
    ms = []
    for row in rows:
        us = [U[int(g.sides.ring[s]) - 1] for s in g.combos.sides[row]]
        ms.append(max(sum(us) + 1, 2 * max(us) + 1))
    assert min(ms) < b.ng  # some combinations really use a smaller grid
    red = _S_on_grid(b, g, Delta, rows, ms)
    scale = np.abs(full).max()
    assert np.abs(red - full).max() < 1e-12 * scale


def test_one_point_fewer_aliases():
    """m = U_1 + U_2 + U_3 admits a wrapped closure for some combination."""
    b, g, Delta, U = _setup()
    rows, ms = [], []
    for row in range(len(g.combos.ntri)):
        us = [U[int(g.sides.ring[s]) - 1] for s in g.combos.sides[row]]
        m = sum(us)
        if 2 * max(us) + 1 <= m and m < b.ng:
            rows.append(row)
            ms.append(m)
        if len(rows) == 40:
            break
    rows = np.array(rows)
    full = triple_sums_fft(g, Delta, rows)
    red = _S_on_grid(b, g, Delta, rows, ms)
    assert np.abs(red - full).max() > 1e-6 * np.abs(full).max()
