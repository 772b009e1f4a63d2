"""GPU checks at the grid sizes of the batched, validation and largest
workloads (N_g = 96, 192, 384, 512), and of the test-support entry points.

* Stored oracle parity at N_g = 96 (the uneven batch's binning, 20 k1 x
  10 mu x 10 t) and N_g = 192, and every l at N_g = 128: expected values
  written by tests/golden/make_golden.py, which runs only the oracle.
* Stage buffers at every size: the Delta planes of the forward FFT against a
  float64 library FFT of the same field, and D (Eq. 9) of sampled grid sides
  of every grid level against the ring's modes folded onto that grid and
  transformed by the library FFT.
* Contraction cells at full size (N_g = 256, 384, 512): S = sum over the
  item's grid of D_A D_B conj(D_C) (Eq. 8 on the reduced grid) of sampled
  work items of every grid level, against float64 sums of the library's own
  D (the contraction alone) and of the reference D (ring sums and
  contraction).
* N_g = 512 binned outputs, which no oracle run reaches, by properties: the
  float32 path against the float64 path, and the z reflection.
* D set directly (bk_debug_set_D): the contraction and binning alone on ring
  sums computed here, against the oracle.
* The graph-replayed estimate against the kernel-by-kernel one, bit for bit.
"""
import os
import sys

import numpy as np
import pytest

from oracle.estimator import estimate
from oracle.geometry import Binning, make_rings
from synth import FieldRecipe, field_digest, make_field

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {2: 1e-11, 1: 1e-5}


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _errors(B, ref):
    nlm = ref.shape[0]
    B, ref = B.reshape(nlm, -1), ref.reshape(nlm, -1)
    assert np.array_equal(np.isnan(B), np.isnan(ref)), "empty-bin pattern differs"
    ok = ~np.isnan(ref)
    return np.array([np.max(np.abs(B[j][ok[j]] - ref[j][ok[j]])) / np.max(np.abs(ref[j][ok[j]])) for j in range(nlm)])


# --- stored oracle values ---------------------------------------------------------


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("name", ["ng96", "ng192", "ng128_all_l"])
def test_stored_oracle_parity(name, prec):
    torch = _torch()
    from paper_2405_14513_amd import bk

    gold = np.load(os.path.join(HERE, "golden", f"oracle_{name}.npz"))
    ng, n_k1, k1_min, k1_max, n_mu, n_t = gold["binning"][:6]
    even = int(gold["binning"][6]) if len(gold["binning"]) > 6 else 1
    rec = gold["recipe"]
    recipe = FieldRecipe(int(rec[0]), n_s=float(rec[1]), f_ng=float(rec[2]), beta=float(rec[3]),
                         sigma_g=float(rec[4]), seed=int(rec[5]))
    _say(f"stored oracle parity {name} prec={prec}")
    delta = make_field(recipe)
    assert field_digest(delta) == str(gold["digest"]), "regenerated field differs from the stored one"
    est = bk.Estimator(bk.make_binning(int(ng), int(n_k1), k1_min, k1_max, int(n_mu), int(n_t), even_l_only=even),
                       prec=prec)
    try:
        s = torch.cuda.current_stream().cuda_stream
        est.load(torch.from_numpy(delta.astype(np.float32) if prec == 1 else delta).cuda(), s)
        est.estimate(s)
        B = est.multipoles()[0]
        assert np.array_equal(est.counts(), gold["counts"])
        assert est.lm_list() == [tuple(x) for x in gold["lms"].tolist()]
    finally:
        est.close()
    err = _errors(B, gold["B"])
    _say(f"  max error per multipole {err.max():.3e}")
    assert err.max() < TOL[prec], err


# --- library-FFT references ----------------------------------------------------------

_RINGS = {}


def _rings(ng):
    if ng not in _RINGS:
        _RINGS[ng] = make_rings(ng)
    return _RINGS[ng]


def _reference_D(torch, Dft, ring_modes, plane, m):
    """Eq. 9 on an m x m grid: the ring's modes of plane `plane` placed at u mod m, forward 2-D FFT."""
    ng = Dft.shape[0]
    ux = torch.from_numpy(ring_modes[:, 0]).to(Dft.device)
    uy = torch.from_numpy(ring_modes[:, 1]).to(Dft.device)
    vals = Dft[ux % ng, uy % ng, plane]
    folded = torch.zeros((m, m), dtype=torch.complex128, device=Dft.device)
    folded.index_put_((ux % m, uy % m), vals, accumulate=True)
    return torch.fft.fft2(folded)


def _field_on_device(torch, ng, seed):
    from synth import make_field_torch

    return make_field_torch(FieldRecipe(ng, n_s=-2.0 if ng != 512 else -1.5, f_ng=0.5, beta=0.5, seed=seed))


SIZES = {  # binning of each size: the workloads' own
    96: (20, 1.0, 32.0, 10, 10),
    192: (20, 1.0, 64.0, 10, 10),
    384: (40, 1.0, 128.0, 12, 12),
    512: (60, 1.0, 512 / 3, 20, 15),
}


def _device_spectrum(torch, field, prec):
    """float64 library FFT of the (rounded) input field, in the plan's units (N^-3/2 DFT)."""
    ng = field.shape[0]
    x = field if prec == 2 else field.to(torch.float32).to(torch.float64)
    return torch.fft.fftn(x) * ng ** -1.5


def _load_estimate(torch, est, field, prec):
    s = torch.cuda.current_stream().cuda_stream
    est.load(field if prec == 2 else field.to(torch.float32).contiguous(), s)
    est.estimate(s)
    torch.cuda.synchronize()


def _check_stage_buffers(torch, bk, est, Dft, prec):
    """Delta planes (K1) and D of sampled grid sides of every grid level (K2)
    of the last estimate against the library-FFT references."""
    ng = Dft.shape[0]
    tol = 1e-13 if prec == 2 else 1e-5
    n2 = ng * ng
    nplanes = bk.bk_debug_get_buffer_size(est.plan, 0) // (n2 * (8 if prec == 1 else 16))
    worst_f = 0.0
    for n in range(nplanes):
        F = torch.from_numpy(bk.bk_debug_read_range(est.plan, 0, prec, n * n2, n2).astype(np.complex128))
        ref = Dft[:, :, n].cpu()
        worst_f = max(worst_f, float((F.reshape(ng, ng) - ref).abs().max() / ref.abs().max()))
    _say(f"  Delta planes: {nplanes}, worst error {worst_f:.2e}")
    assert worst_f < tol
    tab = bk.bk_debug_get_buffer(est.plan, 2, prec).reshape(-1, 3).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(tab[:, 2] ** 2)])
    rings = _rings(ng)
    levels = sorted(set(tab[:, 2].tolist()))
    _say(f"  grid levels {levels}")
    if ng >= 384:
        assert {256, 320, ng} <= set(levels)
    worst_d = 0.0
    for m in levels:
        idx = np.flatnonzero(tab[:, 2] == m)
        pick = sorted(set([idx[0], idx[len(idx) // 2], idx[-1], idx[np.argmax(tab[idx, 0])]]))
        for g in pick:
            r, n, _ = tab[g]
            Dg = bk.bk_debug_read_range(est.plan, 1, prec, int(offs[g]), int(m * m)).astype(np.complex128)
            ref = _reference_D(torch, Dft, rings.modes[r - 1], int(n), int(m)).cpu().numpy().ravel()
            e = np.abs(Dg - ref).max() / np.abs(ref).max()
            worst_d = max(worst_d, e)
            assert e < tol, (r, n, m, e)
    _say(f"  D of sampled grid sides: worst error {worst_d:.2e}")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("ng,prec", [(96, 2), (96, 1), (192, 2), (192, 1), (384, 2)],
                         ids=["ng96-f64", "ng96-f32", "ng192-f64", "ng192-f32", "ng384-f64"])
def test_stage_buffers_every_size(ng, prec):
    """Delta planes (K1) and D of sampled grid sides of every grid level (K2);
    N_g = 384 in float32 and 512 are checked with their contraction cells below."""
    torch = _torch()
    from paper_2405_14513_amd import bk

    _say(f"stage buffers ng={ng} prec={prec}: building the plan")
    field = _field_on_device(torch, ng, seed=31)
    est = bk.Estimator(bk.make_binning(ng, *SIZES[ng]), prec=prec)
    try:
        _load_estimate(torch, est, field, prec)
        _check_stage_buffers(torch, bk, est, _device_spectrum(torch, field, prec), prec)
    finally:
        est.close()


# --- contraction cells at full size ------------------------------------------------


def _decode(bk, plan, prec):
    groups = bk.bk_debug_get_buffer(plan, 4, prec).reshape(-1, 8)
    items = bk.bk_debug_get_buffer(plan, 3, prec).reshape(-1, 144)
    gsides = bk.bk_debug_get_buffer(plan, 5, prec)
    tab = bk.bk_debug_get_buffer(plan, 2, prec).reshape(-1, 3).astype(np.int64)
    return groups, items, gsides, tab


def _check_cells(torch, bk, est, Dft, prec, even):
    """Re S (and Im S for every-l plans) of sampled work items of every grid
    level of the last estimate: against float64 sums of the library's own D
    (the contraction alone, tight bar) and of the reference D (loose bar).
    The bar is relative to the first-order error bound of S from per-side
    relative errors of D."""
    ng = Dft.shape[0]
    groups, items, gsides, tab = _decode(bk, est.plan, prec)
    offs = np.concatenate([[0], np.cumsum(tab[:, 2] ** 2)])
    cells = 512 if even == 0 else 256
    rings = _rings(ng)
    rng = np.random.default_rng(5)
    by_grid = {}
    for gi, gd in enumerate(groups):
        by_grid.setdefault(int(gd[5]), []).append(gi)
    cache_gpu, cache_ref = {}, {}

    def side_pair(g):
        if g not in cache_gpu:
            r, n, m = tab[g]
            Dg = bk.bk_debug_read_range(est.plan, 1, prec, int(offs[g]), int(m * m)).astype(np.complex128)
            cache_gpu[g] = torch.from_numpy(Dg).cuda()
            cache_ref[g] = _reference_D(torch, Dft, rings.modes[r - 1], int(n), int(m)).reshape(-1)
        return cache_gpu[g], cache_ref[g]

    worst_own, worst_ref, checked = 0.0, 0.0, 0
    for m, gl in sorted(by_grid.items()):
        for gi in rng.choice(gl, size=min(2, len(gl)), replace=False):
            gd = groups[gi]
            side_begin, n_sides, item_begin, n_items = (int(v) for v in gd[:4])
            for it in rng.choice(n_items, size=min(2, n_items), replace=False):
                item = item_begin + int(it)
                desc = items[item]
                S = bk.bk_debug_read_range(est.plan, 6, prec, item * cells, cells)
                zero = torch.zeros(m * m, dtype=torch.complex128, device="cuda")

                def D_of(slot):
                    if slot == n_sides:
                        return zero, zero
                    return side_pair(int(gsides[side_begin + slot]) & 0xFFFFFF)

                A = [D_of(int(v)) for v in desc[0:16]]
                C = [D_of(int(v)) for v in desc[64:80]]
                Bs = [D_of(int(v)) for v in desc[128:144]]
                for k in (0, 1):  # 0: the library's own D, 1: reference D
                    PA = torch.stack([a[k] * torch.conj(c[k]) for a, c in zip(A, C)])
                    DB = torch.stack([b[k] for b in Bs])
                    Sref = (PA @ DB.transpose(0, 1).contiguous()).cpu().numpy()  # [pair][column]
                    # first-order bound of the error from per-side relative errors of D
                    aA = torch.stack([a[k].abs() for a in A])
                    aC = torch.stack([c[k].abs() for c in C])
                    aB = torch.stack([b[k].abs() for b in Bs])
                    mA, mC, mB = (t.max(dim=1).values for t in (aA, aC, aB))
                    bound = (mA[:, None] * (aC @ aB.T) + mC[:, None] * (aA @ aB.T)
                             + mB[None, :] * (aA * aC).sum(dim=1)[:, None]).cpu().numpy()
                    got = S[:256].reshape(16, 16)
                    e_re = np.max(np.abs(got - Sref.real) / np.maximum(bound, 1e-300))
                    e = e_re
                    if even == 0:
                        got_im = S[256:512].reshape(16, 16)
                        e = max(e, np.max(np.abs(got_im - Sref.imag) / np.maximum(bound, 1e-300)))
                    if k == 0:
                        worst_own = max(worst_own, float(e))
                    else:
                        worst_ref = max(worst_ref, float(e))
                checked += 1
    _say(f"  {checked} items over grids {sorted(by_grid)}: contraction alone {worst_own:.2e}, "
         f"with reference D {worst_ref:.2e}")
    assert checked >= 2 * len(by_grid)
    assert worst_own < (1e-12 if prec == 2 else 1e-5)
    assert worst_ref < (1e-11 if prec == 2 else 1e-4)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [1, 2], ids=["f32", "f64"])
def test_contraction_cells_ng256(prec):
    torch = _torch()
    from paper_2405_14513_amd import bk

    _say(f"contraction cells ng=256 prec={prec}: building the plan")
    field = _field_on_device(torch, 256, seed=41)
    est = bk.Estimator(bk.make_binning(256, 40, 1.0, 256 / 3, 20, 10), prec=prec)
    try:
        _load_estimate(torch, est, field, prec)
        _check_cells(torch, bk, est, _device_spectrum(torch, field, prec), prec, 1)
    finally:
        est.close()


@pytest.mark.timeout(600)
def test_ng384_float32_every_l():
    """The paper's grid size in float32 with every l: stage buffers and contraction cells."""
    torch = _torch()
    from paper_2405_14513_amd import bk

    _say("ng=384 float32 every l: building the plan")
    field = _field_on_device(torch, 384, seed=41)
    est = bk.Estimator(bk.make_binning(384, *SIZES[384], even_l_only=0), prec=1)
    try:
        _load_estimate(torch, est, field, 1)
        Dft = _device_spectrum(torch, field, 1)
        _check_stage_buffers(torch, bk, est, Dft, 1)
        _check_cells(torch, bk, est, Dft, 1, 0)
    finally:
        est.close()


@pytest.mark.timeout(900)
def test_ng512():
    """N_g = 512, the largest configuration (60 k1 x 20 mu x 15 t bins, every
    l <= 6), in bench.py's launch configuration.  Float32 plan: stage buffers
    and contraction cells against the library-FFT references.  No oracle run
    fits this size for the binned outputs, so properties that hold at any
    size: the float32 path agrees with the float64 path to the float32 bar,
    and under a z reflection of the field the float64 path keeps every even l
    and negates every odd l."""
    torch = _torch()
    from paper_2405_14513_amd import bk

    ng = 512
    binning = bk.make_binning(ng, *SIZES[ng], even_l_only=0)
    field = _field_on_device(torch, ng, seed=7)
    s = torch.cuda.current_stream().cuda_stream
    res = {}
    _say("ng=512: float32 plan")
    est = bk.Estimator(binning, prec=1)
    try:
        _load_estimate(torch, est, field, 1)
        res[(1, "field")] = est.multipoles()[0]
        Dft = _device_spectrum(torch, field, 1)
        _check_stage_buffers(torch, bk, est, Dft, 1)
        _check_cells(torch, bk, est, Dft, 1, 0)
        del Dft
        lms = est.lm_list()
    finally:
        est.close()
    _say("ng=512: float64 plan")
    flip = torch.roll(torch.flip(field, dims=[2]), 1, dims=2).contiguous()
    est = bk.Estimator(binning, prec=2)
    try:
        for name, f in (("field", field), ("flip", flip)):
            est.load(f, s)
            est.estimate(s)
            res[(2, name)] = est.multipoles()[0]
    finally:
        est.close()
    del field, flip
    B64, B32, Bf = res[(2, "field")], res[(1, "field")], res[(2, "flip")]
    nlm = len(lms)
    B64, B32, Bf = B64.reshape(nlm, -1), B32.reshape(nlm, -1), Bf.reshape(nlm, -1)
    assert np.array_equal(np.isnan(B64), np.isnan(B32)) and np.array_equal(np.isnan(B64), np.isnan(Bf))
    worst32, worst_flip = 0.0, 0.0
    for j, (l, _) in enumerate(lms):
        ok = ~np.isnan(B64[j])
        scale = np.max(np.abs(B64[j][ok]))
        assert scale > 0, lms[j]
        worst32 = max(worst32, np.max(np.abs(B32[j][ok] - B64[j][ok])) / scale)
        sign = -1.0 if l % 2 else 1.0
        worst_flip = max(worst_flip, np.max(np.abs(Bf[j][ok] - sign * B64[j][ok])) / scale)
    _say(f"  float32 vs float64 {worst32:.3e}, z reflection {worst_flip:.3e}")
    assert worst32 < 1e-5
    assert worst_flip < 1e-11


# --- D set directly --------------------------------------------------------------


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_set_D_runs_contraction_and_binning(prec):
    """Ring sums computed here with the library FFT, set with bk_debug_set_D:
    the contraction and binning alone reproduce the oracle."""
    torch = _torch()
    from paper_2405_14513_amd import bk

    args = (48, 4, 2.0, 16.0, 6, 5)
    recipe = FieldRecipe(48, n_s=-1.5, f_ng=0.5, beta=1.0, seed=2)
    delta = make_field(recipe)
    ref = estimate(delta, Binning(*args))
    est = bk.Estimator(bk.make_binning(*args), prec=prec)
    try:
        s = torch.cuda.current_stream().cuda_stream
        tab = bk.bk_debug_get_buffer(est.plan, 2, prec).reshape(-1, 3).astype(np.int64)
        Dft = torch.fft.fftn(torch.from_numpy(delta).cuda()) * 48 ** -1.5
        rings = _rings(48)
        parts = [_reference_D(torch, Dft, rings.modes[r - 1], int(n), int(m)).reshape(-1) for r, n, m in tab]
        D = torch.cat(parts).to(torch.complex64 if prec == 1 else torch.complex128).contiguous()
        bk.bk_debug_set_D(est.plan, D.data_ptr(), 1, True, s)
        est.batch = 1
        est.estimate(s)
        B = est.multipoles()[0]
        st = bk.bk_get_stage_times(est.plan)
        assert st[0] < 0.05 and st[1] < 0.05  # no FFT stage ran
        err = _errors(B, ref.B)
        _say(f"set-D prec={prec}: max error per multipole {err.max():.3e}")
        assert err.max() < TOL[prec], err
        # the next estimate without a grid loaded is refused; with one it runs the full path
        with pytest.raises(bk.BkError):
            bk.bk_debug_set_D(est.plan, D.data_ptr(), 2, True, s)  # batch > max_batch
    finally:
        est.close()


# --- graph replay ----------------------------------------------------------------


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_graph_replay_matches_timed_launches(prec):
    """bk_estimate (graph replay) equals bk_estimate_timed bit for bit, over
    several replays with other work and synchronisations between them, across
    a change of batch size (new capture), and stage times average over the
    consecutive timed estimates."""
    torch = _torch()
    from paper_2405_14513_amd import bk

    args = (32, 4, 1.0, 32 / 3, 5, 4)
    fields = np.stack([make_field(FieldRecipe(32, seed=s)) for s in (8, 9)])
    est = bk.Estimator(bk.make_binning(*args), prec=prec, max_batch=2)
    try:
        s = torch.cuda.current_stream().cuda_stream
        t = torch.from_numpy(fields).cuda()
        est.load(t, s)
        est.estimate_timed(s)
        ref = est.multipoles()
        for rep in range(3):
            est.estimate(s)
            torch.cuda.synchronize()
            G = est.multipoles()
            assert np.array_equal(np.isnan(G), np.isnan(ref))
            ok = ~np.isnan(ref)
            assert np.array_equal(G[ok], ref[ok]), f"replay {rep}"
            (torch.randn(1 << 20, device="cuda") * 2).sum().item()
        with pytest.raises(bk.BkError) as e:
            est.stage_times()  # a graph replay records no stage events
        assert e.value.status == bk.BK_ERR_STATE
        for _ in range(3):
            est.estimate_timed(s)
        out = bk.bk_get_stage_times_count(est.plan)
        assert out[4] == 3 and all(v >= 0 for v in out[:4])
        one = t[1:].contiguous()
        est.load(one, s)
        est.estimate(s)
        G1 = est.multipoles()
        ok = ~np.isnan(ref[1])
        assert np.array_equal(G1[0][ok], ref[1][ok])
    finally:
        est.close()
