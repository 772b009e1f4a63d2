"""Pins of the oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a second
formula the paper gives for the same quantity, a closed form, an invariance,
an independent library routine, or a sign the paper states.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import special

from oracle.analytic import continuum_multipole, discrete_prediction, bispectrum_real, kaiser_factor, side_cosines
from oracle.estimator import fourier_field, multipoles, side_D, triple_sums_brute, triple_sums_fft
from oracle.geometry import Binning, make_geometry, make_rings, ring_edges, triangle_counts
from oracle.ylm import assoc_legendre, lm_list, norm_lm, ylm
from synth import FieldRecipe, make_field, plane_wave_field, power_amplitude

C1 = Binning(16, 3, 2.0, 5.0, 5, 3)


@pytest.fixture(scope="module")
def c1_geom():
    return make_geometry(C1)


@pytest.fixture(scope="module")
def c1_field():
    return make_field(FieldRecipe(16, n_s=-2.0, f_ng=0.5, beta=0.5, seed=0))


# --- rings (implementation paragraph of Sec. II) ------------------------------


def _lattice_count_below(r2_num, r2_den):
    """#{(x, y) in Z^2 : x^2 + y^2 < r2_num / r2_den} by counting columns."""
    total = 0
    lim = int(math.isqrt(r2_num // r2_den + 1)) + 1
    for x in range(-lim, lim + 1):
        # largest |y| with x^2 + y^2 < R^2, i.e. y^2 * den < num - x^2 * den
        rem = r2_num - x * x * r2_den
        if rem <= 0:
            continue
        y = math.isqrt((rem - 1) // r2_den) if rem > r2_den else 0
        while (y + 1) ** 2 * r2_den < rem:
            y += 1
        while y > 0 and y * y * r2_den >= rem:
            y -= 1
        total += 2 * y + 1
    return total


@pytest.mark.parametrize("ng", [16, 24, 64, 96, 128])
def test_ring_mode_counts_by_column_counting(ng):
    rings = make_rings(ng)
    edges = ring_edges(ng)
    for r in range(1, len(edges)):
        hi, lo = edges[r], edges[r - 1]
        inside_hi = _lattice_count_below(hi.numerator ** 2, hi.denominator ** 2)
        inside_lo = _lattice_count_below(lo.numerator ** 2, lo.denominator ** 2) if lo > 0 else 0
        assert rings.counts()[r - 1] == inside_hi - inside_lo


def test_ring_schedule_doubles_every_ten_and_caps_at_third():
    e = ring_edges(512)
    widths = [e[i] - e[i - 1] for i in range(1, len(e) - 1)]
    assert widths[:10] == [1] * 10 and widths[10:20] == [2] * 10 and widths[20:30] == [4] * 10
    assert e[-1] == Fraction(512, 3) and len(e) - 1 == 42
    assert len(ring_edges(256)) - 1 == 32 and len(ring_edges(16)) - 1 == 6


def test_ring_counts_n16_by_hand():
    # |u|^2 in [0,1): 1; [1,4): 4+4; [4,9): 4+8+4; [9,16): 4+8+8; [16,25): 4+8+4+8;
    # [25, 28.4): 25 -> 12, 26 -> 8
    assert make_rings(16).counts().tolist() == [1, 8, 16, 20, 24, 20]


def test_mean_radius_small_rings():
    K = make_rings(16).mean_radius
    assert K[0] == 0.0
    assert K[1] == pytest.approx((4 * 1 + 4 * math.sqrt(2)) / 8, rel=1e-15)
    assert K[2] == pytest.approx((4 * 2 + 8 * math.sqrt(5) + 4 * math.sqrt(8)) / 16, rel=1e-15)


# --- triangle counts (Eqs. 10-12) --------------------------------------------


@pytest.mark.parametrize("ng", [16, 32, 48])
def test_ntri_direct_equals_fft_form(ng):
    """Eq. 10 (direct count) equals Eq. 11 (x_perp sum of I I I / N_g^2)."""
    rings = make_rings(ng)
    direct = triangle_counts(rings)
    I = []
    for m in rings.modes:
        mask = np.zeros((ng, ng))
        mask[m[:, 0] % ng, m[:, 1] % ng] = 1.0
        I.append(np.fft.fft2(mask))  # I(r, x) = sum_{u in r} e^{-i u.x}
    I = np.array(I).reshape(len(I), -1)
    via_fft = np.einsum("ax,bx,cx->abc", I, I, I) / ng ** 2
    assert np.max(np.abs(via_fft.imag)) < 1e-6
    assert np.array_equal(np.rint(via_fft.real).astype(np.int64), direct)
    assert np.max(np.abs(via_fft.real - direct)) < 1e-6


def test_ntri_closed_forms():
    ng = 64
    rings = make_rings(ng)
    nt = triangle_counts(rings)
    cnt = rings.counts()
    nr = rings.n_rings
    # ring 1 holds only u = 0: N_tri(1, r, r') = |r| delta_rr'
    assert np.array_equal(nt[0], np.diag(cnt))
    # symmetric under any permutation of the three rings
    for p in [(1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0), (2, 0, 1)]:
        assert np.array_equal(nt, nt.transpose(p))
    # if every u + v stays below N_g/3, every w = -u - v lands in some ring
    edges = ring_edges(ng)
    for r1 in range(nr):
        for r2 in range(nr):
            if edges[r1 + 1] + edges[r2 + 1] <= Fraction(ng, 3):
                assert nt[r1, r2].sum() == cnt[r1] * cnt[r2]
    # total ordered perpendicular triangles at N_g = 16 (hand-checkable size)
    assert triangle_counts(make_rings(16)).sum() == 4645


# --- Y_l^m ---------------------------------------------------------------------


def test_ylm_orthonormal():
    x, wx = np.polynomial.legendre.leggauss(16)
    phi = 2 * np.pi * np.arange(32) / 32
    th = np.arccos(x)
    T, P = np.meshgrid(th, phi, indexing="ij")
    W = wx[:, None] * (2 * np.pi / 32) * np.ones_like(P)
    pairs = [(l, m) for l in range(7) for m in range(-l, l + 1)]
    Y = np.array([ylm(l, m, T, P).ravel() for l, m in pairs])
    G = (Y.conj() * W.ravel()) @ Y.T
    assert np.max(np.abs(G - np.eye(len(pairs)))) < 1e-13


def test_ylm_matches_scipy_and_closed_forms():
    rng = np.random.default_rng(1)
    th = rng.uniform(0, np.pi, 50)
    ph = rng.uniform(0, 2 * np.pi, 50)
    for l in range(9):
        for m in range(-l, l + 1):
            ref = special.sph_harm_y(l, m, th, ph)
            assert np.max(np.abs(ylm(l, m, th, ph) - ref)) < 1e-12
    # Condon-Shortley phase: Y_1^1 = -sqrt(3/(8 pi)) sin(theta) e^{i phi}
    assert np.allclose(ylm(1, 1, th, ph), -math.sqrt(3 / (8 * math.pi)) * np.sin(th) * np.exp(1j * ph))
    assert np.allclose(ylm(2, 2, th, ph), 0.25 * math.sqrt(15 / (2 * math.pi)) * np.sin(th) ** 2 * np.exp(2j * ph))
    assert np.allclose(ylm(2, 0, th, ph), 0.25 * math.sqrt(5 / math.pi) * (3 * np.cos(th) ** 2 - 1))


def test_sixteen_outputs():
    assert len(lm_list(6, 6, True)) == 16
    assert lm_list(6, 6, True)[:4] == [(0, 0), (2, 0), (2, 1), (2, 2)]


# --- Eq. 8 equals Eq. 6 ----------------------------------------------------------


def test_fft_estimator_equals_direct_sum(c1_geom, c1_field):
    Delta = fourier_field(c1_field)
    Tf = triple_sums_fft(c1_geom, Delta)
    Tb, nb = triple_sums_brute(c1_geom, Delta)
    assert len(Tf) == len(c1_geom.combos.ntri) > 400
    assert np.array_equal(nb, c1_geom.combos.ntri)
    assert np.max(np.abs(Tf - Tb)) <= 1e-13 * np.max(np.abs(Tb))


def test_fft_estimator_equals_direct_sum_other_grid():
    b = Binning(12, 2, 2.0, 4.0, 3, 2, box_len=30.0)
    g = make_geometry(b)
    delta = make_field(FieldRecipe(12, box_len=30.0, n_s=-1.5, f_ng=0.5, beta=1.0, seed=3))
    Delta = fourier_field(delta, 30.0)
    Tf = triple_sums_fft(g, Delta)
    Tb, nb = triple_sums_brute(g, Delta)
    assert np.array_equal(nb, g.combos.ntri)
    assert np.max(np.abs(Tf - Tb)) <= 1e-13 * np.max(np.abs(Tb))


def test_side_D_is_masked_dft():
    """Eq. 9 by an explicit sum over the ring's modes at a few x_perp."""
    ng = 16
    delta = make_field(FieldRecipe(ng, seed=5))
    Delta = fourier_field(delta)
    g = make_geometry(C1)
    D = side_D(Delta, g, 3, 2)
    modes = g.rings.modes[2]
    for x, y in [(0, 0), (3, 7), (15, 1)]:
        ref = sum(
            Delta[ux % ng, uy % ng, 2] * np.exp(-2j * np.pi * (ux * x + uy * y) / ng) for ux, uy in modes
        )
        assert abs(D[x, y] - ref) < 1e-12 * max(1.0, abs(ref))


# --- closed-form field: three plane waves ---------------------------------------


def test_three_plane_waves_closed_form():
    ng = 16
    ma, mb = np.array([2, 1, 1]), np.array([-1, 2, -2])
    mc = -(ma + mb)
    waves = [(ma, 0.7, 0.3), (mb, 1.1, -1.2), (mc, 0.9, 2.0)]
    delta = plane_wave_field(ng, waves)
    b = Binning(ng, 3, 2.0, 5.0, 5, 3)
    g = make_geometry(b)
    Delta = fourier_field(delta)
    T = triple_sums_fft(g, Delta)
    vol = float(ng) ** 3
    expect = vol ** 2 * 0.7 * 1.1 * 0.9 * np.exp(1j * (0.3 - 1.2 + 2.0))
    nz = np.flatnonzero(np.abs(T) > 1e-9 * abs(expect))
    assert len(nz) == 2  # the combination and its n -> -n mirror
    vals = sorted(T[nz], key=lambda z: z.imag)
    assert abs(vals[1] - expect) < 1e-10 * abs(expect)
    assert abs(vals[0] - np.conj(expect)) < 1e-10 * abs(expect)
    # the multipoles: only that bin is non-zero and equals 2 w Re(T) / den
    res = multipoles(g, T)
    c = g.combos
    i = nz[0]
    pref = np.array([math.sqrt((2 * l + 1) / (4 * math.pi)) for l, _ in b.lms()])
    Bflat = res.B.reshape(len(pref), -1)
    want = pref * 2 * c.w[i] * expect.real / res.den[:, c.bin[i]]
    assert np.allclose(Bflat[:, c.bin[i]], want, rtol=1e-12, atol=0)
    others = np.ones(b.n_bins, bool)
    others[c.bin[i]] = False
    vals = Bflat[:, others]
    assert np.nanmax(np.abs(vals)) < 1e-9 * np.max(np.abs(want))


# --- odd l: the imaginary part of Eq. 13 (reading in oracle/estimator.py) ---------

C1_ODD = Binning(16, 3, 2.0, 5.0, 5, 3, even_l_only=False)


def _partner_index(geom):
    """For every combination, the index of its n -> -n partner."""
    sides = geom.sides
    key = {}
    trio = geom.combos.sides
    for i, t in enumerate(trio):
        key[tuple(sorted((int(sides.ring[s]), int(sides.plane[s])) for s in t))] = i
    out = np.empty(len(trio), dtype=np.int64)
    for i, t in enumerate(trio):
        out[i] = key[tuple(sorted((int(sides.ring[s]), -int(sides.plane[s])) for s in t))]
    return out


def test_odd_l_weights_flip_between_partners():
    """Partners (every n negated) have p_z -> -p_z and phi -> pi - phi; by the
    parity P_l^m(-x) = (-1)^(l+m) P_l^m(x) and cos(m (pi - phi)) = (-1)^m
    cos(m phi) their weights differ by (-1)^l; the |Y|^2 weights agree."""
    g = make_geometry(C1_ODD)
    part = _partner_index(g)
    sign = np.array([(-1.0) ** l for l, _ in C1_ODD.lms()])
    assert any(l % 2 for l, _ in C1_ODD.lms())
    w, d = g.combos.w, g.combos.d
    assert np.max(np.abs(w[part] - sign * w)) < 1e-13
    assert np.max(np.abs(d[part] - d)) < 1e-13
    # and the bins agree (the sorted side lengths are the same)
    assert np.array_equal(g.combos.bin[part], g.combos.bin)


def test_three_plane_waves_odd_l_closed_form():
    """Odd l of three plane waves: the one bin holds sqrt((2l+1)/4pi) 2 w Im(T)/den
    with T = V^2 A1 A2 A3 e^{i(phi1+phi2+phi3)} on the combination that carries T."""
    ng = 16
    ma, mb = np.array([2, 1, 1]), np.array([-1, 2, -2])
    mc = -(ma + mb)
    waves = [(ma, 0.7, 0.3), (mb, 1.1, -1.2), (mc, 0.9, 2.0)]
    delta = plane_wave_field(ng, waves)
    g = make_geometry(C1_ODD)
    T = triple_sums_fft(g, fourier_field(delta))
    vol = float(ng) ** 3
    expect = vol ** 2 * 0.7 * 1.1 * 0.9 * np.exp(1j * (0.3 - 1.2 + 2.0))
    nz = np.flatnonzero(np.abs(T) > 1e-9 * abs(expect))
    assert len(nz) == 2
    i = nz[np.argmin(np.abs(T[nz] - expect))]
    assert abs(T[i] - expect) < 1e-10 * abs(expect)
    res = multipoles(g, T)
    c = g.combos
    lms = C1_ODD.lms()
    odd = np.array([l % 2 == 1 for l, _ in lms])
    pref = np.array([math.sqrt((2 * l + 1) / (4 * math.pi)) for l, _ in lms])
    Bflat = res.B.reshape(len(lms), -1)
    want = pref * 2 * c.w[i] * np.where(odd, expect.imag, expect.real) / res.den[:, c.bin[i]]
    assert np.max(np.abs(want[odd])) > 0.05 * np.max(np.abs(want))  # odd l really carry signal
    assert np.allclose(Bflat[:, c.bin[i]], want, rtol=1e-12, atol=1e-14 * np.max(np.abs(want)))


def test_z_reflection_flips_odd_l(c1_field):
    """delta(x, y, -z): every combination goes to its partner, so even l keep
    their value and odd l change sign; a z-symmetric field has no odd l."""
    g = make_geometry(C1_ODD)
    odd = np.array([l % 2 == 1 for l, _ in C1_ODD.lms()])
    flip = np.ascontiguousarray(np.roll(c1_field[:, :, ::-1], 1, axis=2))
    r0 = multipoles(g, triple_sums_fft(g, fourier_field(c1_field)))
    r1 = multipoles(g, triple_sums_fft(g, fourier_field(flip)))
    rs = multipoles(g, triple_sums_fft(g, fourier_field(0.5 * (c1_field + flip))))
    ok = np.isfinite(r0.B)
    scale = np.nanmax(np.abs(r0.B))
    B0, B1, Bs = r0.B[ok].reshape(-1), r1.B[ok].reshape(-1), rs.B[ok].reshape(-1)
    oddm = np.broadcast_to(odd[:, None, None, None], r0.B.shape)[ok].reshape(-1)
    assert np.max(np.abs(B0[oddm])) > 1e-3 * scale  # odd l are not zero for this field
    assert np.max(np.abs(B1[~oddm] - B0[~oddm])) < 1e-12 * scale
    assert np.max(np.abs(B1[oddm] + B0[oddm])) < 1e-12 * scale
    assert np.max(np.abs(Bs[oddm])) < 1e-12 * scale


# --- invariances -------------------------------------------------------------------


def test_metamorphic_invariances(c1_geom, c1_field):
    Delta = fourier_field(c1_field)
    T0 = triple_sums_fft(c1_geom, Delta)
    scale = np.max(np.abs(T0))
    # translation by a grid vector
    T1 = triple_sums_fft(c1_geom, fourier_field(np.roll(c1_field, (3, -5, 7), axis=(0, 1, 2))))
    assert np.max(np.abs(T1 - T0)) < 1e-12 * scale
    # 90 degree rotation about z and an x mirror map every ring onto itself
    rot = np.ascontiguousarray(np.rot90(c1_field, k=1, axes=(0, 1)))
    T2 = triple_sums_fft(c1_geom, fourier_field(rot))
    assert np.max(np.abs(T2 - T0)) < 1e-12 * scale
    mir = np.ascontiguousarray(c1_field[::-1])
    T3 = triple_sums_fft(c1_geom, fourier_field(mir))
    assert np.max(np.abs(T3 - T0)) < 1e-12 * scale
    # cubic scaling delta -> a delta
    T4 = triple_sums_fft(c1_geom, fourier_field(2.5 * c1_field))
    assert np.max(np.abs(T4 - 2.5 ** 3 * T0)) < 1e-12 * 2.5 ** 3 * scale
    # z flip: every combination goes to its n -> -n partner, whose T is conj
    flip = np.ascontiguousarray(np.roll(c1_field[:, :, ::-1], 1, axis=2))
    T5 = triple_sums_fft(c1_geom, fourier_field(flip))
    res0 = multipoles(c1_geom, T0)
    res5 = multipoles(c1_geom, T5)
    ok = np.isfinite(res0.B)
    assert np.max(np.abs(res5.B[ok] - res0.B[ok])) < 1e-12 * np.nanmax(np.abs(res0.B))


def test_multipoles_of_conjugate_pairs_are_real(c1_geom, c1_field):
    """Even-l numerators are real: the n -> -n partners carry conj T, same weight."""
    T = triple_sums_fft(c1_geom, fourier_field(c1_field))
    res = multipoles(c1_geom, T)
    assert np.max(np.abs(res.num.imag)) < 1e-12 * np.max(np.abs(res.num.real))


# --- the analytic model (Eqs. 4, 15, 17) -------------------------------------------


def test_continuum_b21_sign_pattern():
    """Sec. III.D: B_2^1 > 0 for mu < t, < 0 for mu > t, ~ 0 at mu = t (beta = 1)."""
    for mu in np.linspace(0.5, 0.99, 8):
        for t in np.linspace(0.5, 1.0, 8):
            if 2 * mu * t < 1.0:
                continue
            v = continuum_multipole(2, 1, mu, t, 1.0).real
            if t - mu > 0.15:
                assert v > 0, (mu, t, v)
            if mu - t > 0.15:
                assert v < 0, (mu, t, v)
    assert abs(continuum_multipole(2, 1, 0.8, 0.8, 1.0).real) < 0.05 * continuum_multipole(0, 0, 0.8, 0.8, 1.0).real
    # magnitude: |B_2^1| a few times smaller than B_0^0 (the paper quotes ~4x)
    assert abs(continuum_multipole(2, 1, 0.95, 0.7, 1.0)) < 0.3 * abs(continuum_multipole(0, 0, 0.95, 0.7, 1.0))


def test_continuum_vanishing_pattern():
    """Eq. 17's angular factor is an even degree-6 polynomial in p: odd l and l > 6 vanish.

    With Eq. 3 every mu_i depends on p_z and p_x only and mu_1 = p_z, so the
    highest power of p_x is 4 and m = 5, 6 vanish as well for this model
    (the paper's count of 16 non-zero multipoles includes l = 6, m = 5, 6).
    """
    mu, t = 0.7, 0.85
    for l in range(0, 9):
        for m in range(0, l + 1):
            v = continuum_multipole(l, m, mu, t, 1.0)
            if l % 2 or l > 6 or m > 4:
                assert abs(v) < 1e-12, (l, m)
            else:
                assert abs(v) > 1e-4, (l, m)
    # beta = 0: only the monopole survives and it equals B_r (Eq. 4 with Y_0^0)
    assert abs(continuum_multipole(0, 0, mu, t, 0.0) - 1.0) < 1e-13
    assert abs(continuum_multipole(2, 1, mu, t, 0.0)) < 1e-13


def test_discrete_prediction_tracks_continuum():
    """[B]_d (estimator's weights) ~ [B]_c (independent quadrature of Eq. 4).

    This ties the oracle's orientation formula (Eq. 3) and Y weights to Eq. 4.
    The two differ by discreteness (Sec. III.C), which is a few percent of the
    monopole at k1 ~ 25-32 k_f away from the squeezed corner.
    """
    b = Binning(96, 1, 25.0, 32.0, 5, 5)
    g = make_geometry(b)
    bd = discrete_prediction(g, 1.0, -2.0, 0.5, 1.0).reshape(len(b.lms()), -1)
    c = g.combos
    k, _ = side_cosines(g)
    br = bispectrum_real(k[:, 0], k[:, 1], k[:, 2], 1.0, -2.0, 0.5)
    nt = c.ntri.astype(float)
    tol = {(0, 0): 0.03, (2, 0): 0.06, (2, 1): 0.06, (2, 2): 0.06, (4, 0): 0.08}
    checked = 0
    for ib in range(b.n_bins):
        sel = c.bin == ib
        if not sel.any():
            continue
        mu_bar = np.sum(c.mu[sel] * nt[sel]) / nt[sel].sum()
        t_bar = np.sum(c.t[sel] * nt[sel]) / nt[sel].sum()
        if mu_bar > 0.85:
            continue  # the squeezed corner is where the paper also sees the largest deviations
        br_bar = np.sum(br[sel] * nt[sel]) / nt[sel].sum()
        mono = continuum_multipole(0, 0, mu_bar, t_bar, 1.0).real
        for j, (l, m) in enumerate(b.lms()):
            if (l, m) not in tol:
                continue
            cont = continuum_multipole(l, m, mu_bar, t_bar, 1.0).real
            assert abs(bd[j, ib] / br_bar - cont) < tol[(l, m)] * mono, (l, m, ib, bd[j, ib] / br_bar, cont)
            checked += 1
    assert checked >= 50


def test_orientation_reproduces_third_side_of_closed_triangles():
    """For exactly closed triangles, p from (mu_1, mu_2) must give p.k3_hat = n_3/k_3.

    The triangle frame has k1_hat = z and k2_hat = (sqrt(1-mu^2), 0, -mu), so
    k3_hat = -(k1 k1_hat + k2 k2_hat)/k3 follows from closure alone; a wrong
    sign or term in p_x breaks the check.  Also |p| = 1 holds without clamping.
    """
    from oracle.geometry import orientation

    rng = np.random.default_rng(7)
    checked = 0
    while checked < 300:
        a = rng.integers(-9, 10, 3).astype(float)
        b_ = rng.integers(-9, 10, 3).astype(float)
        c_ = -(a + b_)
        sides = sorted([a, b_, c_], key=lambda v: -float(v @ v))
        k = [math.sqrt(float(v @ v)) for v in sides]
        if min(k) == 0 or k[0] == k[1] or k[1] == k[2]:
            continue
        mu = -float(sides[0] @ sides[1]) / (k[0] * k[1])
        if abs(mu) > 0.999:
            continue
        px, py, pz, deg = orientation(np.array([sides[0][2]]), np.array([sides[1][2]]), k[0], k[1], mu)
        s = math.sqrt(1 - mu * mu)
        k3hat = -(k[0] * np.array([0.0, 0.0, 1.0]) + k[1] * np.array([s, 0.0, -mu])) / k[2]
        p = np.array([px[0], py[0], pz[0]])
        assert abs(p @ k3hat - sides[2][2] / k[2]) < 1e-12
        assert abs(p @ p - 1.0) < 1e-12
        checked += 1


def test_beta_zero_monopole_is_ntri_weighted_mean():
    b = Binning(32, 4, 3.0, 10.0, 4, 4)
    g = make_geometry(b)
    bd = discrete_prediction(g, 2.0, -2.0, 0.5, 0.0)
    c = g.combos
    k, _ = side_cosines(g)
    br = bispectrum_real(k[:, 0], k[:, 1], k[:, 2], 2.0, -2.0, 0.5)
    num = np.bincount(c.bin, weights=br * c.ntri, minlength=b.n_bins)
    den = np.bincount(c.bin, weights=c.ntri.astype(float), minlength=b.n_bins)
    ok = den > 0
    assert np.allclose(bd[0].ravel()[ok], num[ok] / den[ok], rtol=1e-13)


def test_generator_power_and_variance():
    rec = FieldRecipe(64, n_s=-2.0, f_ng=0.0, beta=0.0, seed=11)
    g = make_field(rec)
    assert abs(np.mean(g)) < 1e-12
    assert 0.3 < np.std(g) < 0.5  # expected sigma_G = 0.4
    # Kaiser: the z-axis modes of delta_s are (1 + beta) times the real-space ones
    r0 = make_field(FieldRecipe(32, beta=0.0, seed=2))
    r1 = make_field(FieldRecipe(32, beta=0.5, seed=2))
    F0, F1 = np.fft.fftn(r0), np.fft.fftn(r1)
    assert np.allclose(F1[0, 0, 1:5], 1.5 * F0[0, 0, 1:5], rtol=1e-12)
    assert np.allclose(F1[1:5, 0, 0], F0[1:5, 0, 0], rtol=1e-12)
    assert power_amplitude(FieldRecipe(16)) > 0
