"""Pins of the oracle's second-level binning and combination enumeration.

* ``_bin_index`` (Eq. 13's intervals) on hand-computed values: linear k1
  shells on [k1_min, k1_max), mu and t linear on [0.5, 1] with the top bin
  closed, flattened as (k1, mu, t).
* Completeness of the enumeration (Sec. II, Step II: every combination of
  three rings and planes): every ordered lattice triangle of a small grid is
  classified into its (ring, plane) cells by code written here, folded into
  its multiset of cells and cut on (k1, mu, t); the resulting set must be the
  oracle's combination list, and the number of ordered triangles of each must
  be its N_tri (Eq. 10) times the number of distinct slot assignments.
* The order of the per-bin triangle count at the paper's validation setup
  (Sec. III.D): the count of closed triangles with k1 >= k2 >= k3 in a bin is
  the phase-space volume 8 pi^2 (int k1^5 dk1) (int int t^2 dt dmu), up to
  lattice discreteness.
"""
import math
import os
from fractions import Fraction
from itertools import permutations

import numpy as np
import pytest

from oracle.geometry import Binning, _bin_index, make_geometry, make_rings, ring_edges

HERE = os.path.dirname(os.path.abspath(__file__))


# --- the second-level bin index -------------------------------------------------


def test_bin_index_by_hand():
    # n_k1 = 4 shells of width 2 on [2, 10); 4 mu bins and 2 t bins of widths 1/8, 1/4
    b = Binning(64, 4, 2.0, 10.0, 4, 2)
    cases = [
        # (k1, mu, t) -> (ik, imu, it)
        ((2.0, 0.5, 0.5), (0, 0, 0)),      # every lower edge opens its bin
        ((3.999, 0.6249, 0.7499), (0, 0, 0)),
        ((4.0, 0.625, 0.75), (1, 1, 1)),   # k1, mu, t exactly on an inner edge: the upper bin
        ((9.999, 0.875, 0.8), (3, 3, 1)),
        ((6.5, 1.0, 1.0), (2, 3, 1)),      # mu = t = 1 fall into the closed top bins
        ((8.0, 0.75, 0.5), (3, 2, 0)),
    ]
    for (k1, mu, t), (ik, imu, it) in cases:
        got = _bin_index(b, np.array([k1]), np.array([mu]), np.array([t]))[0]
        assert got == (ik * 4 + imu) * 2 + it, ((k1, mu, t), got)
    # the flattening order: k1 slowest, t fastest
    got = _bin_index(b, np.array([2.0, 2.0, 4.0]), np.array([0.5, 0.625, 0.5]), np.array([0.75, 0.5, 0.5]))
    assert got.tolist() == [1, 2, 8]


def test_k1_max_is_excluded_and_k1_min_included():
    """k1 = k1_max is outside the last shell; k1 = k1_min is inside the first."""
    b = Binning(16, 3, 2.0, 5.0, 5, 3)
    g = make_geometry(b)
    k1 = g.combos.k1
    assert np.all((k1 >= 2.0) & (k1 < 5.0))
    # the side (ring 1, n = 2) has k = 2 exactly, and combinations with it as
    # the longest side (e.g. with two (ring 2, n = -1) sides) are kept
    assert np.any(k1 == 2.0)


# --- enumeration completeness ------------------------------------------------------


def _ring_of(q, edges):
    """Ring number r with R_{r-1} <= sqrt(q) < R_r (0 if none), in exact arithmetic."""
    out = np.zeros(q.shape, dtype=np.int64)
    for r in range(len(edges) - 1, 0, -1):
        e = edges[r]
        inside = q * e.denominator ** 2 < e.numerator ** 2
        out[inside] = r
    return out


def _brute_cells(binning):
    """Ordered lattice triangles (m1, m2, m3 = -m1 - m2) folded per cell multiset.

    Every mode with |u_perp| < N_g/3 and |n| <= ceil(k1_max) is a candidate;
    the k = 0 cell (ring 1, plane 0) is left out.  Returns a dict
    multiset -> number of ordered triangles, where a multiset is the sorted
    tuple of its three (ring, plane) cells.
    """
    ng = binning.ng
    edges = ring_edges(ng)
    nmax = int(math.ceil(binning.k1_max))
    lim = ng // 3 + 1
    u = np.arange(-lim, lim + 1)
    ux, uy, uz = np.meshgrid(u, u, np.arange(-nmax, nmax + 1), indexing="ij")
    ux, uy, uz = ux.ravel(), uy.ravel(), uz.ravel()
    r = _ring_of(ux * ux + uy * uy, edges)
    keep = (r > 0) & ~((r == 1) & (uz == 0))
    ux, uy, uz, r = ux[keep], uy[keep], uz[keep], r[keep]
    cells = {}
    for i in range(len(ux)):
        wx, wy, wz = -ux[i] - ux, -uy[i] - uy, -uz[i] - uz
        r3 = _ring_of(wx * wx + wy * wy, edges)
        ok = (r3 > 0) & (np.abs(wz) <= nmax) & ~((r3 == 1) & (wz == 0))
        c1 = (int(r[i]), int(uz[i]))
        for rr2, n2, rr3, n3 in zip(r[ok].tolist(), uz[ok].tolist(), r3[ok].tolist(), wz[ok].tolist()):
            key = tuple(sorted((c1, (rr2, n2), (rr3, n3))))
            cells[key] = cells.get(key, 0) + 1
    return cells


def _cut(binning, K, key):
    """(k1, mu, t) of a cell multiset from the mean radii; None when not kept."""
    q = sorted((K[r - 1] * K[r - 1] + float(n) * float(n) for r, n in key), reverse=True)
    k1, k2 = math.sqrt(q[0]), math.sqrt(q[1])
    t = k2 / k1
    mu = min(max(((q[0] + q[1]) - q[2]) / ((2.0 * k1) * k2), -1.0), 1.0)
    if binning.k1_min <= k1 < binning.k1_max and 0.5 <= t <= 1.0 and 0.5 <= mu <= 1.0:
        return k1, mu, t
    return None


@pytest.mark.parametrize(
    "binning",
    [Binning(16, 3, 2.0, 5.0, 5, 3), Binning(12, 2, 2.0, 4.0, 3, 2, box_len=30.0), Binning(16, 2, 1.0, 5.3, 4, 4)],
    ids=["C1", "ng12", "ng16_wide"],
)
def test_enumeration_is_complete(binning):
    g = make_geometry(binning)
    K = g.rings.mean_radius
    # mean radii, recomputed here as plain averages of |u| over each ring's modes
    edges = ring_edges(binning.ng)
    lim = binning.ng // 3 + 1
    u = np.arange(-lim, lim + 1)
    gx, gy = np.meshgrid(u, u, indexing="ij")
    rr = _ring_of(gx * gx + gy * gy, edges)
    for r in range(1, len(edges)):
        assert abs(np.mean(np.sqrt(gx[rr == r] ** 2 + gy[rr == r] ** 2)) - K[r - 1]) < 1e-12

    brute = _brute_cells(binning)
    kept = {key: cnt for key, cnt in brute.items() if _cut(binning, K, key) is not None}

    sides = g.sides
    c = g.combos
    oracle = {}
    for i, trio in enumerate(c.sides):
        key = tuple(sorted((int(sides.ring[s]), int(sides.plane[s])) for s in trio))
        assert key not in oracle, "a cell multiset appears twice"
        oracle[key] = i
    assert set(oracle) == set(kept)
    assert len(kept) > 100
    for key, cnt in kept.items():
        i = oracle[key]
        n_assign = len(set(permutations(key)))
        assert cnt == n_assign * int(c.ntri[i]), key
    # per-bin tally of ordered triangles, one slot assignment per combination
    tally = np.zeros(binning.n_bins, dtype=np.int64)
    for key, cnt in kept.items():
        k1, mu, t = _cut(binning, K, key)
        n_assign = len(set(permutations(key)))
        ik = min(int(math.floor((k1 - binning.k1_min) / ((binning.k1_max - binning.k1_min) / binning.n_k1))),
                 binning.n_k1 - 1)
        imu = min(int(math.floor((mu - 0.5) / (0.5 / binning.n_mu))), binning.n_mu - 1)
        it = min(int(math.floor((t - 0.5) / (0.5 / binning.n_t))), binning.n_t - 1)
        tally[(ik * binning.n_mu + imu) * binning.n_t + it] += cnt // n_assign
    assert np.array_equal(tally, g.bin_counts())


# --- per-bin triangle count against the continuum phase-space volume ---------------


def _continuum_counts(k1_min, k1_max, n):
    """Closed triangles with k1 >= k2 >= k3 per (mu, t) bin of an n x n grid.

    For every k1 vector in the shell (4 pi k1^2 dk1 lattice points per unit
    volume) the k2 vectors with |k2| = t k1 and -cos(k1, k2) = mu fill
    2 pi k1^3 t^2 dt dmu; k3 <= k2 is 2 mu t >= 1.  Integrated with a fine
    midpoint rule in (mu, t).
    """
    radial = 8.0 * math.pi ** 2 * (k1_max ** 6 - k1_min ** 6) / 6.0
    edges = np.linspace(0.5, 1.0, n + 1)
    sub = 200
    out = np.zeros((n, n))
    for i in range(n):
        mu = edges[i] + (np.arange(sub) + 0.5) * (edges[i + 1] - edges[i]) / sub
        for j in range(n):
            t = edges[j] + (np.arange(sub) + 0.5) * (edges[j + 1] - edges[j]) / sub
            M, T = np.meshgrid(mu, t, indexing="ij")
            cell = (edges[i + 1] - edges[i]) * (edges[j + 1] - edges[j]) / sub ** 2
            out[i, j] = np.sum(T ** 2 * (2.0 * M * T >= 1.0)) * cell
    full = np.zeros((n, n), dtype=bool)
    for i in range(n):
        for j in range(n):
            full[i, j] = 2.0 * edges[i] * edges[j] >= 1.0  # the whole bin satisfies 2 mu t >= 1
    return radial * out, full


def test_bin_counts_follow_phase_space_volume():
    """Fresh oracle geometry at N_g = 96, k1 in [24, 30): per-bin N_tri tracks
    the continuum count of triangles (each triangle and its negative counted)."""
    b = Binning(96, 1, 24.0, 30.0, 4, 4)
    g = make_geometry(b)
    counts = g.bin_counts().reshape(4, 4).astype(float)
    cont, full = _continuum_counts(24.0, 30.0, 4)
    ratio = counts[full] / cont[full]
    assert np.all((ratio > 0.85) & (ratio < 1.15)), ratio
    assert 0.95 < counts.sum() / cont.sum() < 1.05


def test_bin_counts_at_the_paper_validation_setup():
    """N_g = 384, L = 215 Mpc, k1 in [2.0, 2.2) Mpc^-1, 12 x 12 (mu, t) bins
    (counts stored by tests/golden/make_validation.py, which runs the oracle).

    Every full bin holds the continuum count to within 10%; the largest
    counts are at t = 1 and they fall with t at every mu, as the paper
    describes (Sec. III.D).  The magnitude is about 1.2e9 per bin, twelve
    times the paper's "order of 1e8" (see the module notes: the count here is
    Eq. 10 as written, one slot assignment per ring/plane combination, both a
    triangle and its negative)."""
    z = np.load(os.path.join(HERE, "golden", "validation_ng384.npz"))
    k1_min, k1_max = z["k1"]
    counts = z["counts_12"][0].astype(float)
    cont, full = _continuum_counts(k1_min, k1_max, 12)
    ratio = counts[full] / cont[full]
    assert np.all((ratio > 0.9) & (ratio < 1.1)), ratio
    assert 0.98 < counts.sum() / cont.sum() < 1.07
    med = np.median(counts[counts > 0])
    assert 5e8 < med < 3e9
    # largest at t = 1 (L isosceles); within each mu row of full bins, N_tri grows with t
    assert np.argmax(counts.max(axis=0)) == 11
    for i in range(12):
        row = counts[i][full[i]]
        assert np.all(np.diff(row) > -0.1 * row[:-1]), (i, row)


def test_several_binnings_equal_separate_runs():
    """The oracle's multi-resolution streaming (one T per combination, binned
    under every binning) equals one plain estimate per binning."""
    from oracle.estimator import estimate, estimate_streaming_binnings
    from synth import FieldRecipe, make_field

    delta = make_field(FieldRecipe(24, n_s=-2.0, f_ng=0.5, beta=0.5, seed=3))
    bs = [Binning(24, 2, 2.0, 8.0, 3, 3), Binning(24, 1, 2.0, 8.0, 5, 2), Binning(24, 3, 2.0, 8.0, 2, 4)]
    multi = estimate_streaming_binnings(delta, bs, workers=1, chunks=5)
    for b, got in zip(bs, multi):
        ref = estimate(delta, b)
        assert np.array_equal(got.counts, ref.counts)
        ok = ~np.isnan(ref.B)
        assert np.array_equal(~np.isnan(got.B), ok)
        assert ok.any()
        scale = np.max(np.abs(ref.B[ok]))
        assert np.max(np.abs(got.B[ok] - ref.B[ok])) < 1e-12 * scale
    with pytest.raises(ValueError):
        estimate_streaming_binnings(delta, [bs[0], Binning(24, 2, 2.0, 7.0, 3, 3)])


def test_bin_sampled_streaming_equals_the_full_estimate():
    """Restricting the streaming sums to some bins (and the plane triples that
    can reach them) leaves those bins exactly as the full estimate has them."""
    from oracle.estimator import estimate, estimate_streaming_binnings
    from synth import FieldRecipe, make_field

    delta = make_field(FieldRecipe(24, n_s=-2.0, f_ng=0.5, beta=0.5, seed=3))
    b = Binning(24, 3, 2.0, 8.0, 3, 3)
    ref = estimate(delta, b)
    bins = np.arange(9)  # the lowest k1 shell, [2, 4): every side has k < 4
    got = estimate_streaming_binnings(delta, [b], bins=bins, plane_filter=lambda pt: max(abs(n) for n in pt) < 4.0)[0]
    B = got.B.reshape(len(got.lms), -1)[:, bins]
    R = ref.B.reshape(len(ref.lms), -1)[:, bins]
    ok = ~np.isnan(R)
    assert ok.any() and np.array_equal(~np.isnan(B), ok)
    assert np.max(np.abs(B[ok] - R[ok])) < 1e-12 * np.max(np.abs(R[ok]))
    assert np.array_equal(got.counts.ravel()[bins], ref.counts.ravel()[bins])
