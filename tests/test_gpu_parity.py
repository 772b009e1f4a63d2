"""GPU parity: the HIP path (through the C ABI) against the float64 oracle.

Error metric per multipole (l, m): max over non-empty bins of |B_gpu - B_oracle|
divided by max over bins of |B_oracle| (a per-bin ratio is unbounded where a
multipole crosses zero).  Bars: 1e-11 for the float64 path, 1e-5 for float32.
Triangle counts must be identical and empty bins NaN on both sides.
"""
import sys

import numpy as np
import pytest

from oracle.estimator import estimate, fourier_field, multipoles, triple_sums_fft
from oracle.geometry import Binning, make_geometry
from synth import FieldRecipe, make_field, plane_wave_field

pytestmark = pytest.mark.gpu

TOL = {2: 1e-11, 1: 1e-5}


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def per_multipole_error(B, ref):
    nlm = ref.shape[0]
    B = B.reshape(nlm, -1)
    ref = ref.reshape(nlm, -1)
    assert np.array_equal(np.isnan(B), np.isnan(ref)), "empty-bin pattern differs"
    ok = ~np.isnan(ref)
    errs = []
    for j in range(nlm):
        scale = np.max(np.abs(ref[j][ok[j]])) if ok[j].any() else 0.0
        diff = np.max(np.abs(B[j][ok[j]] - ref[j][ok[j]])) if ok[j].any() else 0.0
        errs.append(diff / scale if scale > 0 else diff)
    return np.array(errs)


_ORACLE_CACHE = {}


def oracle_result(args, recipe, even=True):
    key = (args, recipe, even)
    if key not in _ORACLE_CACHE:
        b = Binning(*args[:6], box_len=args[6] if len(args) > 6 else None, even_l_only=even)
        delta = make_field(recipe)
        _ORACLE_CACHE[key] = (b, delta, estimate(delta, b))
    return _ORACLE_CACHE[key]


def run_gpu(args, delta, prec, batch_fields=None, as_f32=False, device_input=True, even=True):
    torch = _torch()
    from paper_2405_14513_amd import bk

    binning = bk.make_binning(*args[:6], box_len=args[6] if len(args) > 6 else 0.0, even_l_only=int(even))
    fields = [delta] if batch_fields is None else batch_fields
    arr = np.stack(fields).astype(np.float32 if as_f32 else np.float64)
    est = bk.Estimator(binning, prec=prec, max_batch=len(fields))
    try:
        if device_input:
            t = torch.from_numpy(arr).cuda()
            stream = torch.cuda.current_stream().cuda_stream
            est.load(t, stream)
            est.estimate(stream)
        else:
            est.load(arr)
            est.estimate()
        B = est.multipoles()
        counts = est.counts()
        lms = est.lm_list()
    finally:
        est.close()
    return B, counts, lms


CASES = [
    ((16, 3, 2.0, 5.0, 5, 3), FieldRecipe(16, n_s=-2.0, f_ng=0.5, beta=0.5, seed=0)),
    ((32, 4, 1.0, 32 / 3, 5, 4), FieldRecipe(32, n_s=-2.0, f_ng=0.5, beta=0.5, seed=1)),
    ((48, 4, 2.0, 16.0, 6, 5), FieldRecipe(48, n_s=-1.5, f_ng=0.5, beta=1.0, seed=2)),
    ((64, 6, 1.0, 64 / 3, 8, 6), FieldRecipe(64, n_s=-2.0, f_ng=0.5, beta=0.5, seed=3)),
    ((24, 3, 1.0, 8.0, 4, 4, 37.5), FieldRecipe(24, box_len=37.5, n_s=-2.0, f_ng=0.5, beta=0.5, seed=4)),
]


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("case", range(len(CASES)), ids=[f"ng{c[0][0]}" for c in CASES])
def test_parity_against_oracle(case, prec):
    args, recipe = CASES[case]
    _say(f"parity case ng={args[0]} prec={prec}")
    b, delta, ref = oracle_result(args, recipe)
    B, counts, lms = run_gpu(args, delta, prec)
    assert lms == b.lms()
    assert np.array_equal(counts, ref.counts)
    err = per_multipole_error(B[0], ref.B)
    _say(f"  max error per multipole {err.max():.3e}")
    assert err.max() < TOL[prec], err


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("case", [0, 1, 2, 4], ids=[f"ng{CASES[i][0][0]}" for i in (0, 1, 2, 4)])
def test_odd_l_parity(case, prec):
    """All l up to 6 (odd l from Im S, the imaginary part of Eq. 13) against the oracle."""
    args, recipe = CASES[case]
    _say(f"odd-l parity ng={args[0]} prec={prec}")
    b, delta, ref = oracle_result(args, recipe, even=False)
    B, counts, lms = run_gpu(args, delta, prec, even=False)
    assert lms == b.lms() and any(l % 2 for l, _ in lms)
    assert np.array_equal(counts, ref.counts)
    err = per_multipole_error(B[0], ref.B)
    _say(f"  max error per multipole {err.max():.3e}")
    assert err.max() < TOL[prec], err


WORK_SHAPES = {"items1": {"BK_K3_ITEMS": "1"}, "pairs32": {"BK_K3_PAIRS": "32"},
               "pairs64": {"BK_K3_PAIRS": "64"}, "sides48": {"BK_K3_SIDES": "48"}}


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("shape", list(WORK_SHAPES))
def test_other_work_item_shapes(shape, prec, monkeypatch):
    """The contraction's other work-item shapes against the oracle: one 16-pair
    item per wave, items of two or four row tiles sharing their slot-B reads,
    and a small staged-side cap (many workgroups of few items); the default is
    two 16-pair items per wave."""
    args, recipe = CASES[3]
    even = shape != "pairs32"  # one shape also takes the Im S path (odd l)
    _say(f"work item shape {shape}, ng={args[0]} prec={prec} even_l_only={even}")
    b, delta, ref = oracle_result(args, recipe, even=even)
    for k, v in WORK_SHAPES[shape].items():
        monkeypatch.setenv(k, v)
    B, counts, lms = run_gpu(args, delta, prec, even=even)
    assert np.array_equal(counts, ref.counts)
    err = per_multipole_error(B[0], ref.B)
    _say(f"  max error per multipole {err.max():.3e}")
    assert err.max() < TOL[prec], err


def test_brute_force_small_grid_float64():
    """C1 (N_g = 16) against the direct triangle sum of Eq. 6."""
    args, recipe = CASES[0]
    b = Binning(*args)
    delta = make_field(recipe)
    ref = estimate(delta, b, method="brute")
    B, counts, _ = run_gpu(args, delta, 2)
    assert np.array_equal(counts, ref.counts)
    assert per_multipole_error(B[0], ref.B).max() < 1e-11


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_batched_fields_match_single(prec):
    args, _ = CASES[1]
    fields = [make_field(FieldRecipe(32, seed=s)) for s in (5, 6, 7)]
    Bb, _, _ = run_gpu(args, None, prec, batch_fields=fields)
    for i, f in enumerate(fields):
        Bs, _, _ = run_gpu(args, f, prec)
        ok = ~np.isnan(Bs[0])
        assert np.array_equal(np.isnan(Bb[i]), np.isnan(Bs[0]))
        assert np.max(np.abs(Bb[i][ok] - Bs[0][ok])) == 0.0


def test_float32_input_and_host_pointer():
    args, recipe = CASES[1]
    b, delta, ref = oracle_result(args, recipe)
    B, _, _ = run_gpu(args, delta, 1, as_f32=True, device_input=False)
    # input rounding to float32 adds ~1e-7 relative per cell
    assert per_multipole_error(B[0], ref.B).max() < 1e-5


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_three_plane_waves(prec):
    ng = 16
    ma, mb = np.array([2, 1, 1]), np.array([-1, 2, -2])
    waves = [(ma, 0.7, 0.3), (mb, 1.1, -1.2), (-(ma + mb), 0.9, 2.0)]
    delta = plane_wave_field(ng, waves)
    args = (16, 3, 2.0, 5.0, 5, 3)
    b = Binning(*args)
    g = make_geometry(b)
    ref = multipoles(g, triple_sums_fft(g, fourier_field(delta)))
    B, _, _ = run_gpu(args, delta, prec)
    ok = ~np.isnan(ref.B)
    scale = np.nanmax(np.abs(ref.B))
    assert np.max(np.abs(B[0][ok] - ref.B[ok])) < (1e-11 if prec == 2 else 1e-5) * scale


def test_error_paths():
    torch = _torch()
    from paper_2405_14513_amd import bk

    binning = bk.make_binning(16, 3, 2.0, 5.0, 5, 3)
    plan = bk.bk_plan_create(binning, bk.BK_F64, 0, 1)
    try:
        with pytest.raises(bk.BkError) as e:
            bk.bk_estimate(plan, 0)
        assert e.value.status == bk.BK_ERR_STATE
        with pytest.raises(bk.BkError) as e:
            bk.bk_get_multipoles(plan, 1)
        assert e.value.status == bk.BK_ERR_STATE
        t = torch.zeros((2, 16, 16, 16), dtype=torch.float64, device="cuda")
        with pytest.raises(bk.BkError) as e:
            bk.bk_load_grid(plan, t.data_ptr(), bk.BK_F64, 2, True, 0)  # batch > max_batch
        assert e.value.status == bk.BK_ERR_ARG
        bk.bk_load_grid(plan, t.data_ptr(), bk.BK_F64, 1, True, 0)
        bk.bk_estimate(plan, 0)
        with pytest.raises(bk.BkError) as e:
            bk.bk_get_multipoles(plan, 1, cap=3)
        assert e.value.status == bk.BK_ERR_SIZE
        B = bk.bk_get_multipoles(plan, 1)
        # a zero field gives zero in every non-empty bin
        assert np.nanmax(np.abs(B)) == 0.0
    finally:
        bk.bk_plan_destroy(plan)
    with pytest.raises(bk.BkError) as e:
        bk.bk_plan_create(bk.make_binning(16, 3, 2.0, 5.0, 5, 3), 7, 0, 1)
    assert e.value.status == bk.BK_ERR_ARG


@pytest.mark.parametrize("env", [{"BK_K3_ITEMS": "3"}, {"BK_K3_PAIRS": "32", "BK_K3_ITEMS": "2"},
                                 {"BK_K3_PAIRS": "48"}, {"BK_K3_SIDES": "0"}, {"BK_K3_SIDES": "255"}])
def test_invalid_work_item_shape_is_rejected(env, monkeypatch):
    _torch()
    from paper_2405_14513_amd import bk

    for k, v in env.items():
        monkeypatch.setenv(k, v)
    with pytest.raises(bk.BkError) as e:
        bk.bk_plan_create(bk.make_binning(16, 3, 2.0, 5.0, 5, 3), bk.BK_F32, 0, 1)
    assert e.value.status == bk.BK_ERR_ARG


def test_device_memory_cap_reports_oom(monkeypatch):
    _torch()
    from paper_2405_14513_amd import bk

    monkeypatch.setenv("BK_MAX_DEVICE_BYTES", "1000")
    with pytest.raises(bk.BkError) as e:
        bk.bk_plan_create(bk.make_binning(16, 3, 2.0, 5.0, 5, 3), bk.BK_F64, 0, 1)
    assert e.value.status == bk.BK_ERR_OOM


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_mfma_lane_layout(prec):
    """The contraction kernel's result layout: register k of lane l holds
    C[row][l % 16] with row = 4k + l/16 (float64) or 4(l/16) + k (float32)."""
    _torch()
    from paper_2405_14513_amd import bk

    P = bk.bk_debug_mfma_probe(prec)
    for lane in range(64):
        for k in range(4):
            col, kq = lane % 16, lane // 16
            row = 4 * k + kq if prec == 2 else 4 * kq + k
            want = row + 16 * col if col < 4 else 0
            assert P[lane, k] == want, (lane, k, P[lane, k], want)


def side_D_on_grid(Delta, geom, ring, plane, m):
    """Eq. 9 evaluated on an m x m grid: the ring's modes placed at u mod m."""
    ng = Delta.shape[0]
    modes = geom.rings.modes[ring - 1]
    folded = np.zeros((m, m), dtype=np.complex128)
    np.add.at(folded, (modes[:, 0] % m, modes[:, 1] % m), Delta[modes[:, 0] % ng, modes[:, 1] % ng, plane % ng])
    return np.fft.fft2(folded)


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_stage_buffers_match_oracle(prec):
    """Delta planes (K1) and ring sums D (K2, Eq. 9) against numpy's FFT."""
    torch = _torch()
    from oracle.estimator import side_D
    from paper_2405_14513_amd import bk

    args, recipe = CASES[2]  # N_g = 48 exercises the radix-3 stage
    ng = args[0]
    b, delta, _ = oracle_result(args, recipe)
    g = make_geometry(b)
    Dl = fourier_field(delta, b.box_len)
    scale = ng ** -1.5
    est = bk.Estimator(bk.make_binning(*args), prec=prec)
    try:
        t = torch.from_numpy(delta).cuda()
        s = torch.cuda.current_stream().cuda_stream
        est.load(t, s)
        est.estimate(s)
        F = bk.bk_debug_get_buffer(est.plan, 0, prec)
        nkeep = F.size // (ng * ng)
        F = F.reshape(nkeep, ng, ng)
        ref = np.transpose(Dl[:, :, :nkeep], (2, 0, 1)) * scale
        tol = 1e-14 if prec == 2 else 2e-6
        assert np.abs(F - ref).max() < tol * np.abs(ref).max()
        D = bk.bk_debug_get_buffer(est.plan, 1, prec)
        tab = bk.bk_debug_get_buffer(est.plan, 2, prec).reshape(-1, 3)
        assert D.size == int((tab[:, 2].astype(np.int64) ** 2).sum())
        stored = {(int(r), int(n)) for r, n in zip(g.sides.ring, g.sides.plane) if n >= 0}
        assert {(int(r), int(n)) for r, n, _ in tab} <= stored
        assert set(tab[:, 2].tolist()) <= {16, 24, 32, 40, 48} and 40 in set(tab[:, 2].tolist())  # radix-5 level
        off = 0
        for r, n, m in tab:
            Dm = D[off:off + m * m].reshape(m, m)
            off += m * m
            if m == ng:
                Dref = side_D(Dl, g, int(r), int(n)) * scale
            else:
                Dref = side_D_on_grid(Dl, g, int(r), int(n), int(m)) * scale
            assert np.abs(Dm - Dref).max() < tol * max(np.abs(Dref).max(), 1e-300), (r, n, m)
    finally:
        est.close()


@pytest.mark.parametrize("prec", [2, 1])
def test_autotuned_plan_matches_oracle(prec):
    """Every tile choice the tuner tries ends in a correct estimate; the tuned
    plan, and a second plan picking the choice up from the cache, stay within
    the parity bar, with identical triangle counts."""
    torch = _torch()
    from paper_2405_14513_amd import bk

    args, recipe = CASES[2]
    b, delta, ref = oracle_result(args, recipe)
    binning = bk.make_binning(*args)
    stream = torch.cuda.current_stream().cuda_stream
    t = torch.from_numpy(delta).cuda()
    _say(f"autotune N_g=48 prec={prec}")
    est = bk.Estimator(binning, prec=prec)
    est2 = None
    try:
        est.load(t, stream)
        choices = est.autotune(stream)
        assert choices[0] in (2, 4, 8, 16) and choices[1] in (2, 4, 8, 16) and choices[2] in (16, 32, 64)
        err_tuned = per_multipole_error(est.multipoles()[0], ref.B)
        est.estimate(stream)
        err = per_multipole_error(est.multipoles()[0], ref.B)
        assert np.array_equal(est.counts(), ref.counts)
        assert err_tuned.max() < TOL[prec], err_tuned
        assert err.max() < TOL[prec], err
        est2 = bk.Estimator(binning, prec=prec)
        est2.load(t, stream)
        est2.estimate(stream)
        err2 = per_multipole_error(est2.multipoles()[0], ref.B)
        assert err2.max() < TOL[prec], err2
    finally:
        est.close()
        if est2 is not None:
            est2.close()
    with pytest.raises(bk.BkError) as e:
        fresh = bk.Estimator(binning, prec=prec)
        try:
            fresh.autotune(stream)
        finally:
            fresh.close()
    assert e.value.status == bk.BK_ERR_STATE


EDGE_CASES = [
    # smallest grid: two rings beyond the zero ring, k1 up to N_g/3
    ("ng8", dict(ng=8, n_k1=2, k1_min=1.0, k1_max=8 / 3, n_mu=3, n_t=2), FieldRecipe(8, seed=21)),
    # l_max = 12 (49 outputs: the 64-lane binning path)
    ("lmax12", dict(ng=24, n_k1=2, k1_min=3.0, k1_max=8.0, n_mu=3, n_t=3, l_max=12, m_max=12),
     FieldRecipe(24, n_s=-1.5, f_ng=0.5, beta=1.0, seed=22)),
    # m_max < l_max (13 outputs)
    ("mmax2", dict(ng=24, n_k1=2, k1_min=3.0, k1_max=8.0, n_mu=3, n_t=3, l_max=8, m_max=2),
     FieldRecipe(24, n_s=-2.0, f_ng=0.5, beta=0.5, seed=23)),
    # every l <= 8 (45 outputs: the 64-lane binning path with odd-l lanes)
    ("lmax8_all", dict(ng=24, n_k1=2, k1_min=3.0, k1_max=8.0, n_mu=3, n_t=3, l_max=8, m_max=8, even=False),
     FieldRecipe(24, n_s=-1.5, f_ng=0.5, beta=1.0, seed=25)),
    # fine (mu, t) bins at a small grid: many empty bins (NaN pattern)
    ("empty", dict(ng=16, n_k1=3, k1_min=2.5, k1_max=5.0, n_mu=9, n_t=9),
     FieldRecipe(16, n_s=-2.0, f_ng=0.5, beta=0.5, seed=24)),
]


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("case", range(len(EDGE_CASES)), ids=[c[0] for c in EDGE_CASES])
def test_edge_case_parity(case, prec):
    """Degenerate and boundary configurations against the oracle."""
    torch = _torch()
    from paper_2405_14513_amd import bk

    name, kw, recipe = EDGE_CASES[case]
    _say(f"edge case {name} prec={prec}")
    even = kw.get("even", True)
    b = Binning(kw["ng"], kw["n_k1"], kw["k1_min"], kw["k1_max"], kw["n_mu"], kw["n_t"],
                l_max=kw.get("l_max", 6), m_max=kw.get("m_max", 6), even_l_only=even)
    delta = make_field(recipe)
    ref = estimate(delta, b)
    est = bk.Estimator(bk.make_binning(kw["ng"], kw["n_k1"], kw["k1_min"], kw["k1_max"], kw["n_mu"], kw["n_t"],
                                       l_max=kw.get("l_max", 6), m_max=kw.get("m_max", 6), even_l_only=int(even)),
                       prec=prec)
    try:
        s = torch.cuda.current_stream().cuda_stream
        est.load(torch.from_numpy(delta).cuda(), s)
        est.estimate(s)
        assert est.lm_list() == b.lms()
        assert np.array_equal(est.counts(), ref.counts)
        err = per_multipole_error(est.multipoles()[0], ref.B)
        assert err.max() < TOL[prec], err
        if name == "empty":
            assert np.isnan(ref.B).any() and (~np.isnan(ref.B)).any()
    finally:
        est.close()
