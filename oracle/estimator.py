"""Oracle bispectrum-multipole estimator, float64, CPU.

Test infrastructure only: nothing outside ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py`` may import this package.

Two independent ways to get the first-level sum of every combination
c = ((r1, n1), (r2, n2), (r3, n3)):

* ``triple_sums_brute`` -- the direct triangle sum of Eq. 6: every ordered
  pair of grid modes (m1, m2) with m3 = -m1 - m2 is classified into its three
  (ring, plane) cells and Delta(m1) Delta(m2) Delta(m3) is added to that
  ordered cell triple.  O(N_g^6); tiny grids only.
* ``triple_sums_fft`` -- Eq. 8 with D from Eq. 9, each D being a 2-D FFT of
  one ring-masked k_parallel plane; the x_perp sum of D1 D2 D3 is done with a
  matrix product.  Negative planes are transformed directly (no symmetry used).

Both return T(c) = B_hat(c) N_tri(c) = (1/V) sum_{u,v,w} Delta Delta Delta
delta_K(u+v+w) = (1/(V N_g^2)) sum_x D D D, the quantity that enters the
numerator of Eq. 13.  ``multipoles`` then accumulates Eq. 13:
    num_lm[bin] += w_lm(c) T(c),  den_lm[bin] += d_lm(c) N_tri(c),
    count[bin] += N_tri(c),      B_lm = sqrt((2l+1)/(4 pi)) num/den,
with NaN for bins that receive no combination.

Reading for odd l (the paper shows even l only): a combination c and its
partner with every n negated carry conjugate sums, T(c-bar) = conj T(c) for a
real field, and mirror-averaged weights of opposite sign for odd l
(p_z -> -p_z and phi -> pi - phi give (-1)^l), so num_lm is real for even l
and imaginary for odd l.  The reported B_lm is Re(num)/den for even l and
Im(num)/den for odd l (times the prefactor); the other part vanishes
identically.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .geometry import Binning, Geometry, make_geometry


def fourier_field(delta: np.ndarray, box_len: float | None = None) -> np.ndarray:
    """Delta(m) = (V / N_g^3) sum_x delta(x) e^{-2 pi i m.x / N_g} (Sec. II)."""
    ng = delta.shape[0]
    length = float(ng) if box_len is None else float(box_len)
    return (length ** 3 / ng ** 3) * np.fft.fftn(np.asarray(delta, dtype=np.float64))


def side_D(Delta: np.ndarray, geom: Geometry, ring: int, plane: int) -> np.ndarray:
    """D(r, n, x_perp) = sum_{u in ring r} Delta(u, n) e^{-2 pi i u.x / N_g} (Eq. 9)."""
    ng = Delta.shape[0]
    modes = geom.rings.modes[ring - 1]
    masked = np.zeros((ng, ng), dtype=np.complex128)
    ix, iy = modes[:, 0] % ng, modes[:, 1] % ng
    masked[ix, iy] = Delta[ix, iy, plane % ng]
    return np.fft.fft2(masked)


def triple_sums_fft(geom: Geometry, Delta: np.ndarray, rows=None) -> np.ndarray:
    """T(c) for the kept combinations (or the subset ``rows``) via Eq. 8."""
    ng = Delta.shape[0]
    combos = geom.combos
    sel = np.arange(len(combos.ntri)) if rows is None else np.asarray(rows)
    out = np.zeros(len(sel), dtype=np.complex128)
    if not len(sel):
        return out
    ring = geom.sides.ring
    plane = geom.sides.plane
    trio = combos.sides[sel]
    cache = {}

    def D(side):
        if side not in cache:
            cache[side] = side_D(Delta, geom, int(ring[side]), int(plane[side])).ravel()
        return cache[side]

    # group rows by (first side): one matrix product per group
    order = np.lexsort((trio[:, 2], trio[:, 1], trio[:, 0]))
    first = trio[order, 0]
    starts = np.flatnonzero(np.r_[True, first[1:] != first[:-1]])
    ends = np.r_[starts[1:], len(order)]
    for s0, s1 in zip(starts, ends):
        rows_g = order[s0:s1]
        a = D(int(first[s0]))
        bsides = np.unique(trio[rows_g, 1])
        csides = np.unique(trio[rows_g, 2])
        ab = a[None, :] * np.stack([D(int(s)) for s in bsides])
        cm = np.stack([D(int(s)) for s in csides])
        full = ab @ cm.T  # [b, c] = sum_x D_a D_b D_c
        bi = np.searchsorted(bsides, trio[rows_g, 1])
        ci = np.searchsorted(csides, trio[rows_g, 2])
        out[rows_g] = full[bi, ci]
    return out / (geom.binning.volume * ng * ng)


def _side_of_modes(geom: Geometry, mx, my, mz):
    """Side index of each 3-D mode, or -1 when it lies in no kept side."""
    grid_off = 3 * geom.rings.label_radius
    from .geometry import ring_label_grid

    grid, off = ring_label_grid(geom.rings)
    assert off == grid_off
    inside = (np.abs(mx) <= off) & (np.abs(my) <= off)
    r = np.zeros(mx.shape, dtype=np.int64)
    r[inside] = grid[mx[inside] + off, my[inside] + off]
    out = np.full(mx.shape, -1, dtype=np.int64)
    for (rr, nn), idx in geom.sides.index.items():
        out[(r == rr) & (mz == nn)] = idx
    return out


def triple_sums_brute(geom: Geometry, Delta: np.ndarray):
    """T(c) and N_tri(c) by the direct triangle sum of Eq. 6 (O(N_g^6)).

    Returns (T, ntri) for every kept combination, in its slot order.
    """
    ng = Delta.shape[0]
    f = np.fft.fftfreq(ng, d=1.0 / ng).round().astype(np.int64)
    mx, my, mz = np.meshgrid(f, f, f, indexing="ij")
    mx, my, mz = mx.ravel(), my.ravel(), mz.ravel()
    side = _side_of_modes(geom, mx, my, mz)
    keep = side >= 0
    mx, my, mz, side = mx[keep], my[keep], mz[keep], side[keep]
    val = Delta[mx % ng, my % ng, mz % ng]
    nsides = len(geom.sides.ring)
    acc = {}
    cnt = {}
    for i in range(len(mx)):
        # every partner m2; m3 = -m1 - m2 must also land in a side
        x3, y3, z3 = -mx[i] - mx, -my[i] - my, -mz[i] - mz
        s3 = _side_of_modes(geom, x3, y3, z3)
        ok = s3 >= 0
        if not ok.any():
            continue
        v3 = Delta[x3[ok] % ng, y3[ok] % ng, z3[ok] % ng]
        key = (side[i] * nsides + side[ok]) * nsides + s3[ok]
        prod = val[i] * val[ok] * v3
        uk, inv = np.unique(key, return_inverse=True)
        sums = np.zeros(len(uk), dtype=np.complex128)
        np.add.at(sums, inv, prod)
        counts = np.bincount(inv, minlength=len(uk))
        for k, s, c in zip(uk.tolist(), sums.tolist(), counts.tolist()):
            acc[k] = acc.get(k, 0.0) + s
            cnt[k] = cnt.get(k, 0) + c
    trio = geom.combos.sides
    keys = (trio[:, 0] * nsides + trio[:, 1]) * nsides + trio[:, 2]
    T = np.array([acc.get(int(k), 0.0) for k in keys], dtype=np.complex128) / geom.binning.volume
    ntri = np.array([cnt.get(int(k), 0) for k in keys], dtype=np.int64)
    return T, ntri


@dataclass
class Multipoles:
    lms: list
    B: np.ndarray  # (n_lm, n_k1, n_mu, n_t), NaN where empty
    counts: np.ndarray  # (n_k1, n_mu, n_t) int64, sum of N_tri
    num: np.ndarray  # (n_lm, n_bins) complex
    den: np.ndarray  # (n_lm, n_bins)


def _finish(lms, num, den):
    """sqrt((2l+1)/(4 pi)) num/den: the real part for even l, the imaginary
    part for odd l (the other vanishes, see the module notes)."""
    pref = np.array([math.sqrt((2 * l + 1) / (4.0 * math.pi)) for l, _ in lms])
    odd = np.array([l % 2 == 1 for l, _ in lms])
    part = np.where(odd[:, None], num.imag, num.real)
    with np.errstate(invalid="ignore", divide="ignore"):
        return pref[:, None] * part / den


def multipoles(geom: Geometry, T: np.ndarray) -> Multipoles:
    """Second-level binning of Eq. 13, accumulated per combination."""
    b = geom.binning
    lms = b.lms()
    c = geom.combos
    nb = b.n_bins
    num = np.zeros((len(lms), nb), dtype=np.complex128)
    den = np.zeros((len(lms), nb))
    for j in range(len(lms)):
        np.add.at(num[j], c.bin, c.w[:, j] * T)
        np.add.at(den[j], c.bin, c.d[:, j] * c.ntri.astype(np.float64))
    counts = np.zeros(nb, dtype=np.int64)
    np.add.at(counts, c.bin, c.ntri)
    B = _finish(lms, num, den)
    B[:, counts == 0] = np.nan
    B[den == 0.0] = np.nan
    shape = (len(lms), b.n_k1, b.n_mu, b.n_t)
    return Multipoles(lms, B.reshape(shape), counts.reshape(shape[1:]), num, den)


def estimate(delta: np.ndarray, binning: Binning, method: str = "fft", geom: Geometry | None = None) -> Multipoles:
    """All requested B_l^m of one gridded field (the paper's two-step estimator)."""
    geom = make_geometry(binning) if geom is None else geom
    Delta = fourier_field(delta, binning.box_len)
    if method == "fft":
        T = triple_sums_fft(geom, Delta)
    elif method == "brute":
        T, _ = triple_sums_brute(geom, Delta)
    else:
        raise ValueError(method)
    return multipoles(geom, T)


def _stream_chunk(task):
    """Worker: Eq. 8 sums and Eq. 13 accumulators for one set of plane triples."""
    delta, binnings, rings, ntri, sides, triples, bins = task
    return stream_plane_triples_binnings(delta, binnings, rings, ntri, sides, triples, bins)[0]


def stream_plane_triples(delta, binning, rings, ntri, sides, triples):
    """Eq. 8 sums and Eq. 13 accumulators (num, den, counts) over the given
    plane triples, plus the number of combinations visited."""
    parts, n_visited = stream_plane_triples_binnings(delta, [binning], rings, ntri, sides, triples)
    return parts[0] + (n_visited,)


def _same_combinations(binnings):
    """The kept combinations depend on the k1 range, the grid and the (l, m)
    list only; the bin counts decide nothing but the bin index."""
    b0 = binnings[0]
    for b in binnings[1:]:
        if (b.ng, b.k1_min, b.k1_max, b.length, b.l_max, b.m_max, b.even_l_only) != (
                b0.ng, b0.k1_min, b0.k1_max, b0.length, b0.l_max, b0.m_max, b0.even_l_only):
            raise ValueError("binnings may differ in n_k1, n_mu and n_t only")


def stream_plane_triples_binnings(delta, binnings, rings, ntri, sides, triples, bins=None):
    """As ``stream_plane_triples`` for several second-level binnings of the
    same combinations: each combination's T is computed once and added to the
    bin it falls in under every binning.  With ``bins`` (flat bin indices of
    the first binning), only the combinations in those bins are summed, so
    only those bins are complete.  Returns ([(num, den, counts) per binning],
    combinations visited)."""
    from .geometry import Combos, Geometry, _bin_index, combos_for_planes

    _same_combinations(binnings)
    binning = binnings[0]
    n_visited = 0
    nlm = len(binning.lms())
    acc = [(np.zeros((nlm, b.n_bins), dtype=np.complex128), np.zeros((nlm, b.n_bins)),
            np.zeros(b.n_bins, dtype=np.int64)) for b in binnings]
    Delta = fourier_field(delta, binning.box_len)
    for pt in triples:
        res = combos_for_planes(rings, ntri, sides, binning, *pt)
        if res is None:
            continue
        combos = Combos(*res)
        if bins is not None:
            keep = np.isin(combos.bin, bins)
            if not keep.any():
                continue
            combos = Combos(*(a[keep] for a in res))
        n_visited += len(combos.ntri)
        geom = Geometry(binning, rings, ntri, sides, combos)
        T = triple_sums_fft(geom, Delta)
        for b, (num, den, counts) in zip(binnings, acc):
            idx = _bin_index(b, combos.k1, combos.mu, combos.t)
            for j in range(nlm):
                np.add.at(num[j], idx, combos.w[:, j] * T)
                np.add.at(den[j], idx, combos.d[:, j] * combos.ntri.astype(np.float64))
            np.add.at(counts, idx, combos.ntri)
    return acc, n_visited


def estimate_streaming(delta: np.ndarray, binning: Binning, workers: int = 1, chunks: int = 64) -> Multipoles:
    """Same result as ``estimate`` without holding every combination at once.

    Follows the paper's implementation note (end of Sec. II): the first-level
    estimates are never stored; each one's contribution to the numerator and
    denominator of Eq. 13 is accumulated as soon as it is computed.  Plane
    triples are split into ``chunks`` groups, optionally over ``workers``
    processes; the partial sums are added in chunk order.
    """
    return estimate_streaming_binnings(delta, [binning], workers, chunks)[0]


def estimate_streaming_binnings(delta: np.ndarray, binnings, workers: int = 1, chunks: int = 64, bins=None,
                                plane_filter=None) -> list:
    """``estimate_streaming`` for several second-level binnings (Eq. 13 at
    several (mu, t) resolutions, Sec. III.D) that differ in their bin counts
    only: one Multipoles per binning, each equal to a separate run.

    Sampling a grid too large for a full run: ``bins`` restricts the sums to
    the combinations of those bins of the first binning (the other bins come
    out incomplete), and ``plane_filter`` (a predicate on plane triples) skips
    triples that cannot reach them."""
    from .geometry import make_rings, make_sides, plane_triples, triangle_counts

    binning = binnings[0]
    _same_combinations(binnings)
    rings = make_rings(binning.ng)
    ntri = triangle_counts(rings)
    sides = make_sides(rings, binning)
    triples = plane_triples(int(math.ceil(binning.k1_max)))
    if plane_filter is not None:
        triples = [pt for pt in triples if plane_filter(pt)]
    groups = [triples[i::chunks] for i in range(chunks)]
    bins = None if bins is None else np.asarray(bins, dtype=np.int64)
    tasks = [(delta, list(binnings), rings, ntri, sides, g, bins) for g in groups if g]
    if workers > 1:
        import multiprocessing as mp

        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_stream_chunk, tasks, chunksize=1)
    else:
        parts = [_stream_chunk(t) for t in tasks]
    lms = binning.lms()
    out = []
    for ib, b in enumerate(binnings):
        nb = b.n_bins
        num = np.zeros((len(lms), nb), dtype=np.complex128)
        den = np.zeros((len(lms), nb))
        counts = np.zeros(nb, dtype=np.int64)
        for part in parts:
            pnum, pden, pc = part[ib]
            num += pnum
            den += pden
            counts += pc
        B = _finish(lms, num, den)
        B[:, counts == 0] = np.nan
        B[den == 0.0] = np.nan
        shape = (len(lms), b.n_k1, b.n_mu, b.n_t)
        out.append(Multipoles(lms, B.reshape(shape), counts.reshape(shape[1:]), num, den))
    return out
