"""Oracle geometry: rings, sides, triangle counts and ring/plane combinations.

Test infrastructure only: nothing outside ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py`` may import this package.

Everything here follows Sec. II of the paper (the plane x annular-ring binning
of Fig. 1, Eqs. 2, 3, 10 and the implementation paragraph on ring widths),
with the readings below where the paper is silent.  Wave vectors are integer
lattice vectors (units of k_f = 2 pi / L); the line of sight is z.

Readings (the paper does not fix these):
* ring edges R_0 = 0, R_r = R_{r-1} + 2^floor((r-1)/10), the last edge clipped
  to N_g/3; membership is half-open, R_{r-1} <= |u| < R_r, so every mode obeys
  the strict |u| < N_g/3 (three such components can never wrap mod N_g);
* the "mean radius" of a ring is the average of |u| over its lattice modes,
  accumulated in ascending |u|^2 order (so any other implementation that sums
  in that order gets the same float64 bits);
* a side is a (ring, plane) cell (r, n) with mean-value k^2 = K_r^2 + n^2; the
  k = 0 side (ring 1, n = 0) is excluded;
* a combination is an unordered multiset of three sides with n1 + n2 + n3 = 0
  and N_tri > 0; it is kept when k1 is in [k1_min, k1_max) and mu, t are in
  [0.5, 1] (Eq. 2 on the sorted mean values, mu clamped to [-1, 1]);
* the orientation p follows Eq. 3 with p_z = mu1 and p_x from mu2, and
  p_y = +sqrt(max(0, 1 - p_z^2 - p_x^2)).  Each ring combination holds both
  mirror images of every triangle, so Y* is replaced by its mirror average
  N_lm P_l^m(p_z) cos(m phi).  Labellings of sides whose k are exactly equal
  are averaged.  If sqrt(1 - mu^2) < 1e-12 the azimuth is undefined and only
  m = 0 keeps a weight.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from fractions import Fraction
from itertools import permutations

import numpy as np

from .ylm import assoc_legendre, lm_list, norm_lm

DEGENERATE_S = 1e-12


@dataclass(frozen=True)
class Binning:
    """Second-level (k1, mu, t) bins and the multipoles to output (Eq. 13).

    k1 limits are in units of k_f = 2 pi / L.  mu and t bins are linear on
    [0.5, 1] with the top bin closed.
    """

    ng: int
    n_k1: int
    k1_min: float
    k1_max: float
    n_mu: int
    n_t: int
    box_len: float | None = None
    l_max: int = 6
    m_max: int = 6
    even_l_only: bool = True

    @property
    def length(self) -> float:
        return float(self.ng) if self.box_len is None else float(self.box_len)

    @property
    def volume(self) -> float:
        return self.length ** 3

    @property
    def n_bins(self) -> int:
        return self.n_k1 * self.n_mu * self.n_t

    def lms(self):
        return lm_list(self.l_max, self.m_max, self.even_l_only)


def ring_edges(ng: int) -> list:
    """Edges R_0..R_Nr as exact fractions (paper: widths 2^floor((r-1)/10))."""
    cap = Fraction(ng, 3)
    edges = [Fraction(0)]
    r = 1
    while edges[-1] < cap:
        nxt = edges[-1] + 2 ** ((r - 1) // 10)
        edges.append(min(Fraction(nxt), cap))
        r += 1
    return edges


def _below(q: int, edge: Fraction) -> bool:
    """|u| < edge for |u|^2 = q, decided in exact integers."""
    return q * edge.denominator ** 2 < edge.numerator ** 2


@dataclass
class Rings:
    ng: int
    edges: list
    modes: list  # modes[r-1] = int array (count, 2) of (ux, uy)
    mean_radius: np.ndarray  # K_r, float64, index r-1
    label_radius: int  # all modes satisfy |ux|, |uy| <= label_radius

    @property
    def n_rings(self) -> int:
        return len(self.modes)

    def counts(self) -> np.ndarray:
        return np.array([len(m) for m in self.modes], dtype=np.int64)


def make_rings(ng: int) -> Rings:
    edges = ring_edges(ng)
    lim = ng // 3 + 1
    modes = [[] for _ in range(len(edges) - 1)]
    shells = [dict() for _ in range(len(edges) - 1)]  # q -> count, per ring
    for ux in range(-lim, lim + 1):
        for uy in range(-lim, lim + 1):
            q = ux * ux + uy * uy
            for r in range(1, len(edges)):
                if not _below(q, edges[r - 1]) and _below(q, edges[r]):
                    modes[r - 1].append((ux, uy))
                    shells[r - 1][q] = shells[r - 1].get(q, 0) + 1
                    break
    mean = np.zeros(len(modes))
    for i, sh in enumerate(shells):
        if not sh:
            raise ValueError(f"ring {i + 1} of N_g={ng} holds no lattice mode")
        acc = 0.0
        for q in sorted(sh):
            acc += float(sh[q]) * math.sqrt(q)
        mean[i] = acc / float(sum(sh.values()))
    return Rings(ng, edges, [np.array(m, dtype=np.int64) for m in modes], mean, lim)


def ring_label_grid(rings: Rings) -> tuple:
    """2-D array L[ux + off, uy + off] = ring number (0 outside every ring)."""
    off = 3 * rings.label_radius
    size = 2 * off + 1
    grid = np.zeros((size, size), dtype=np.int64)
    for r, m in enumerate(rings.modes, start=1):
        grid[m[:, 0] + off, m[:, 1] + off] = r
    return grid, off


def triangle_counts(rings: Rings) -> np.ndarray:
    """N_tri(r1, r2, r3) of Eq. 10 by direct counting (exact integers).

    N_tri = #{(u, v): u in {r1}, v in {r2}, w = -u - v in {r3}}; returned as an
    int64 array indexed [r1-1, r2-1, r3-1].  It does not depend on the planes.
    """
    nr = rings.n_rings
    grid, off = ring_label_grid(rings)
    allm = np.concatenate(rings.modes)
    lab = np.concatenate([np.full(len(m), r, dtype=np.int64) for r, m in enumerate(rings.modes, start=1)])
    out = np.zeros((nr + 1, nr + 1, nr + 1), dtype=np.int64)
    for (ux, uy), r1 in zip(allm, lab):
        wx = -ux - allm[:, 0] + off
        wy = -uy - allm[:, 1] + off
        r3 = grid[wx, wy]
        keep = r3 > 0
        idx = lab[keep] * (nr + 1) + r3[keep]
        out[r1] += np.bincount(idx, minlength=(nr + 1) ** 2).reshape(nr + 1, nr + 1)
    return out[1:, 1:, 1:]


@dataclass
class Sides:
    """(ring, plane) cells with mean-value k < k1_max, k = 0 excluded."""

    ring: np.ndarray  # 1-based ring number
    plane: np.ndarray  # signed k_parallel index n
    ksq: np.ndarray  # K_r^2 + n^2
    index: dict = field(default_factory=dict)  # (r, n) -> position


def make_sides(rings: Rings, binning: Binning) -> Sides:
    ring, plane, ksq = [], [], []
    nmax = int(math.ceil(binning.k1_max))
    for n in range(-nmax, nmax + 1):
        for r in range(1, rings.n_rings + 1):
            if r == 1 and n == 0:
                continue
            kk = rings.mean_radius[r - 1]
            q = kk * kk + float(n) * float(n)
            if math.sqrt(q) < binning.k1_max:
                ring.append(r)
                plane.append(n)
                ksq.append(q)
    s = Sides(np.array(ring, dtype=np.int64), np.array(plane, dtype=np.int64), np.array(ksq))
    s.index = {(int(r), int(n)): i for i, (r, n) in enumerate(zip(s.ring, s.plane))}
    return s


@dataclass
class Combos:
    """Kept combinations, one row each (unordered multisets of sides)."""

    sides: np.ndarray  # (C, 3) side indices, slot order n1 <= n2 <= n3
    ntri: np.ndarray  # (C,) int64
    k1: np.ndarray
    mu: np.ndarray
    t: np.ndarray
    bin: np.ndarray  # flat (ik, imu, it) index
    w: np.ndarray  # (C, n_lm) mirror-averaged Re Y weights
    d: np.ndarray  # (C, n_lm) |Y|^2 weights


def orientation(n_sorted_1, n_sorted_2, k1, k2, mu):
    """p = (p_x, p_y, p_z) of Eq. 3 from the first two sides' LoS cosines.

    mu_1 = n_1 / k1 = p_z and mu_2 = n_2 / k2 = -mu p_z + sqrt(1 - mu^2) p_x;
    p_y >= 0 completes the unit vector (clamped at 0).  Also returns the
    mask of degenerate (collinear, sqrt(1 - mu^2) < 1e-12) triangles, whose
    p_x is set to 0.
    """
    mu1 = n_sorted_1 / k1
    mu2 = n_sorted_2 / k2
    s = np.sqrt(1.0 - mu * mu)
    degenerate = s < DEGENERATE_S
    s_safe = np.where(degenerate, 1.0, s)
    px = np.where(degenerate, 0.0, (mu2 + mu * mu1) / s_safe)
    py = np.sqrt(np.maximum((1.0 - mu1 * mu1) - px * px, 0.0))
    return px, py, mu1, degenerate


def _weights(lms, n_sorted_1, n_sorted_2, k1, k2, mu):
    """w_lm and d_lm for one labelling (arrays over combinations), Eq. 3."""
    px, py, mu1, degenerate = orientation(n_sorted_1, n_sorted_2, k1, k2, mu)
    phi = np.arctan2(py, px)
    w = np.zeros((len(mu1), len(lms)))
    d = np.zeros((len(mu1), len(lms)))
    for j, (l, m) in enumerate(lms):
        y = norm_lm(l, m) * assoc_legendre(l, m, mu1)
        w[:, j] = np.where(degenerate, y if m == 0 else 0.0, y * np.cos(m * phi))
        d[:, j] = y * y
    return w, d


def _bin_index(binning: Binning, k1, mu, t):
    dk = (binning.k1_max - binning.k1_min) / binning.n_k1
    ik = np.minimum(np.floor((k1 - binning.k1_min) / dk), binning.n_k1 - 1).astype(np.int64)
    dmu = 0.5 / binning.n_mu
    imu = np.minimum(np.floor((mu - 0.5) / dmu), binning.n_mu - 1).astype(np.int64)
    dt = 0.5 / binning.n_t
    it = np.minimum(np.floor((t - 0.5) / dt), binning.n_t - 1).astype(np.int64)
    return (ik * binning.n_mu + imu) * binning.n_t + it


def combos_for_planes(rings, ntri_table, sides, binning, n1, n2, n3):
    """Kept combinations whose sides lie on planes n1 <= n2 <= n3 (sum 0)."""
    def on(n):
        return np.nonzero(sides.plane == n)[0]

    s1, s2, s3 = on(n1), on(n2), on(n3)
    if not (len(s1) and len(s2) and len(s3)):
        return None
    a, b, c = np.meshgrid(s1, s2, s3, indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    keep = np.ones(len(a), dtype=bool)
    if n1 == n2:
        keep &= sides.ring[a] <= sides.ring[b]
    if n2 == n3:
        keep &= sides.ring[b] <= sides.ring[c]
    a, b, c = a[keep], b[keep], c[keep]
    nt = ntri_table[sides.ring[a] - 1, sides.ring[b] - 1, sides.ring[c] - 1]
    keep = nt > 0
    a, b, c, nt = a[keep], b[keep], c[keep], nt[keep]
    if not len(a):
        return None

    trio = np.stack([a, b, c], axis=1)
    q = sides.ksq[trio]
    qs = -np.sort(-q, axis=1)  # descending values
    k1 = np.sqrt(qs[:, 0])
    k2 = np.sqrt(qs[:, 1])
    t = k2 / k1
    mu = ((qs[:, 0] + qs[:, 1]) - qs[:, 2]) / ((2.0 * k1) * k2)
    mu = np.minimum(np.maximum(mu, -1.0), 1.0)
    keep = (k1 >= binning.k1_min) & (k1 < binning.k1_max) & (t >= 0.5) & (t <= 1.0) & (mu >= 0.5) & (mu <= 1.0)
    trio, nt, q, k1, k2, t, mu = trio[keep], nt[keep], q[keep], k1[keep], k2[keep], t[keep], mu[keep]
    if not len(trio):
        return None

    lms = binning.lms()
    nplane = sides.plane[trio].astype(np.float64)
    wsum = np.zeros((len(trio), len(lms)))
    dsum = np.zeros((len(trio), len(lms)))
    nlab = np.zeros(len(trio))
    for p in permutations(range(3)):
        ok = (q[:, p[0]] >= q[:, p[1]]) & (q[:, p[1]] >= q[:, p[2]])
        if not ok.any():
            continue
        w, d = _weights(lms, nplane[:, p[0]], nplane[:, p[1]], k1, k2, mu)
        wsum += np.where(ok[:, None], w, 0.0)
        dsum += np.where(ok[:, None], d, 0.0)
        nlab += ok
    return trio, nt, k1, mu, t, _bin_index(binning, k1, mu, t), wsum / nlab[:, None], dsum / nlab[:, None]


def plane_triples(nmax: int):
    """All (n1, n2, n3) with n1 <= n2 <= n3, n1 + n2 + n3 = 0, |n| <= nmax."""
    out = []
    for n1 in range(-nmax, 1):
        for n2 in range(n1, nmax + 1):
            n3 = -n1 - n2
            if n3 < n2 or n3 > nmax:
                continue
            out.append((n1, n2, n3))
    return out


@dataclass
class Geometry:
    binning: Binning
    rings: Rings
    ntri_table: np.ndarray
    sides: Sides
    combos: Combos

    def bin_counts(self) -> np.ndarray:
        """Sum of N_tri over the kept combinations of each (k1, mu, t) bin."""
        return _int_bincount(self.combos.bin, self.combos.ntri, self.binning.n_bins)


def _int_bincount(idx, vals, n):
    out = np.zeros(n, dtype=np.int64)
    np.add.at(out, idx, vals)
    return out


def make_geometry(binning: Binning, plane_filter=None) -> Geometry:
    """Rings, N_tri, sides and every kept combination for one binning.

    ``plane_filter`` (optional) restricts the plane triples visited; it is
    used only to sample large grids.
    """
    if binning.k1_max > binning.ng / 3.0:
        raise ValueError("k1_max must not exceed N_g/3")
    rings = make_rings(binning.ng)
    ntri = triangle_counts(rings)
    sides = make_sides(rings, binning)
    nmax = int(math.ceil(binning.k1_max))
    parts = []
    for pt in plane_triples(nmax):
        if plane_filter is not None and not plane_filter(pt):
            continue
        res = combos_for_planes(rings, ntri, sides, binning, *pt)
        if res is not None:
            parts.append(res)
    n_lm = len(binning.lms())
    if parts:
        cols = list(zip(*parts))
        combos = Combos(
            np.concatenate(cols[0]),
            np.concatenate(cols[1]),
            np.concatenate(cols[2]),
            np.concatenate(cols[3]),
            np.concatenate(cols[4]),
            np.concatenate(cols[5]),
            np.concatenate(cols[6]),
            np.concatenate(cols[7]),
        )
    else:
        e = np.zeros(0)
        combos = Combos(np.zeros((0, 3), np.int64), np.zeros(0, np.int64), e, e, e, np.zeros(0, np.int64),
                        np.zeros((0, n_lm)), np.zeros((0, n_lm)))
    return Geometry(binning, rings, ntri, sides, combos)
