"""Full-size parity: the N_g = 128 and N_g = 256 workloads, in the launch
configuration bench.py times, against stored float64 oracle values.

tests/golden/oracle_ng<N>.npz was written by tests/golden/make_golden.py,
which calls only the oracle; the field is regenerated here from its seed and
checked against the stored SHA-256 before use.
"""
import os

import numpy as np
import pytest

from synth import FieldRecipe, field_digest, make_field

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
WORKLOADS = {
    128: (20, 1.0, 128 / 3, 10, 10),
    256: (40, 1.0, 256 / 3, 20, 10),
}


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("ng", [128, 256])
def test_fullsize_against_stored_oracle(ng, prec):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_14513_amd import bk

    print(f"full-size parity ng={ng} prec={prec}", flush=True)
    gold = np.load(os.path.join(HERE, "golden", f"oracle_ng{ng}.npz"))
    delta = make_field(FieldRecipe(ng, n_s=-2.0, f_ng=0.5, beta=0.5, seed=0))
    assert field_digest(delta) == str(gold["digest"]), "regenerated field differs from the stored one"
    est = bk.Estimator(bk.make_binning(ng, *WORKLOADS[ng]), prec=prec)
    try:
        arr = delta.astype(np.float32) if prec == 1 else delta
        t = torch.from_numpy(arr).cuda()
        s = torch.cuda.current_stream().cuda_stream
        est.load(t, s)
        est.estimate(s)
        B = est.multipoles()[0]
        counts = est.counts()
        lms = est.lm_list()
    finally:
        est.close()
    assert [tuple(x) for x in gold["lms"].tolist()] == lms
    assert np.array_equal(counts, gold["counts"])
    ref = gold["B"]
    assert np.array_equal(np.isnan(B), np.isnan(ref))
    nlm = ref.shape[0]
    Bf, rf = B.reshape(nlm, -1), ref.reshape(nlm, -1)
    ok = ~np.isnan(rf)
    err = np.array([np.max(np.abs(Bf[j][ok[j]] - rf[j][ok[j]])) / np.max(np.abs(rf[j][ok[j]])) for j in range(nlm)])
    print(f"  max error per multipole {err.max():.3e}", flush=True)
    # float32: input rounded to float32, float32 FFTs and products, float64 sums
    assert err.max() < (1e-11 if prec == 2 else 1e-5), err


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("ng", [128, 256])
def test_fullsize_every_l(ng, prec):
    """Every l at full size: the even l of an every-l plan equal the stored
    even-l oracle values, and under a z reflection of the field the odd l
    (Im S) change sign while the even l stay, as they must (the reflection maps
    every combination to its n -> -n partner)."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_14513_amd import bk

    print(f"full-size every-l ng={ng} prec={prec}", flush=True)
    gold = np.load(os.path.join(HERE, "golden", f"oracle_ng{ng}.npz"))
    delta = make_field(FieldRecipe(ng, n_s=-2.0, f_ng=0.5, beta=0.5, seed=0))
    assert field_digest(delta) == str(gold["digest"]), "regenerated field differs from the stored one"
    flip = np.ascontiguousarray(np.roll(delta[:, :, ::-1], 1, axis=2))
    est = bk.Estimator(bk.make_binning(ng, *WORKLOADS[ng], even_l_only=0), prec=prec)
    out = []
    try:
        s = torch.cuda.current_stream().cuda_stream
        for field in (delta, flip):
            t = torch.from_numpy(field.astype(np.float32) if prec == 1 else field).cuda()
            est.load(t, s)
            est.estimate(s)
            out.append(est.multipoles()[0])
        lms = est.lm_list()
        counts = est.counts()
    finally:
        est.close()
    tol = 1e-11 if prec == 2 else 1e-5
    assert np.array_equal(counts, gold["counts"])
    even = [j for j, (l, _) in enumerate(lms) if l % 2 == 0]
    odd = [j for j, (l, _) in enumerate(lms) if l % 2 == 1]
    assert [lms[j] for j in even] == [tuple(x) for x in gold["lms"].tolist()]
    B, Bf = out[0].reshape(len(lms), -1), out[1].reshape(len(lms), -1)
    ref = gold["B"].reshape(len(even), -1)
    ok = ~np.isnan(ref)
    for i, j in enumerate(even):
        scale = np.max(np.abs(ref[i][ok[i]]))
        assert np.max(np.abs(B[j][ok[i]] - ref[i][ok[i]])) < tol * scale, lms[j]
        assert np.max(np.abs(Bf[j][ok[i]] - ref[i][ok[i]])) < tol * scale, lms[j]
    mono = np.max(np.abs(ref[0][ok[0]]))
    worst = 0.0
    for j in odd:
        okj = ~np.isnan(B[j])
        scale = np.max(np.abs(B[j][okj]))
        assert scale > 1e-6 * mono, lms[j]  # odd l carry signal in a finite realisation
        worst = max(worst, np.max(np.abs(Bf[j][okj] + B[j][okj])) / scale)
    print(f"  odd-l reflection residual {worst:.3e}", flush=True)
    assert worst < tol


@pytest.fixture(scope="module")
def val384_field():
    gold = np.load(os.path.join(HERE, "golden", "oracle_val384.npz"))
    ng, n_s, f_ng, beta, _, seed, box = gold["recipe"]
    print("validation-setup field: generating N_g = 384 on the host", flush=True)
    delta = make_field(FieldRecipe(int(ng), box_len=float(box), n_s=float(n_s), f_ng=float(f_ng), beta=float(beta),
                                   seed=int(seed)))
    assert field_digest(delta) == str(gold["digest"]), "regenerated field differs from the stored one"
    return gold, delta


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_validation_setup_against_stored_oracle(val384_field, prec):
    """The paper's validation configuration (N_g = 384, L = 215 Mpc,
    k1 = 2.1 +- 0.1 Mpc^-1, 12 x 12 (mu, t) bins, l <= 6) on one realisation,
    element by element against the stored float64 oracle, through a
    three-resolution plan (12 x 12, 8 x 8, 6 x 6) whose first resolution is
    the stored binning."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_14513_amd import bk

    gold, delta = val384_field
    ng, n_k1, k1_min, k1_max, n_mu, n_t, even, box = gold["binning"]
    print(f"validation-setup parity prec={prec}", flush=True)
    b = bk.make_binning(int(ng), int(n_k1), float(k1_min), float(k1_max), int(n_mu), int(n_t), box_len=float(box),
                        even_l_only=int(even))
    est = bk.Estimator(b, prec=prec, extra_bins=[(1, 8, 8), (1, 6, 6)])
    try:
        t = torch.from_numpy(delta.astype(np.float32) if prec == 1 else delta).cuda()
        s = torch.cuda.current_stream().cuda_stream
        est.load(t, s)
        est.estimate(s)
        B = est.multipoles(0)[0]
        counts = est.counts(0)
        lms = est.lm_list()
    finally:
        est.close()
    assert [tuple(x) for x in gold["lms"].tolist()] == lms
    assert np.array_equal(counts, gold["counts"])
    ref = gold["B"]
    assert np.array_equal(np.isnan(B), np.isnan(ref))
    nlm = ref.shape[0]
    Bf, rf = B.reshape(nlm, -1), ref.reshape(nlm, -1)
    ok = ~np.isnan(rf)
    err = np.array([np.max(np.abs(Bf[j][ok[j]] - rf[j][ok[j]])) / np.max(np.abs(rf[j][ok[j]])) for j in range(nlm)])
    print(f"  max error per multipole {err.max():.3e}", flush=True)
    assert err.max() < (1e-11 if prec == 2 else 1e-5), err


@pytest.fixture(scope="module")
def ng512_field():
    gold = np.load(os.path.join(HERE, "golden", "oracle_ng512_lowk.npz"))
    ng, n_s, f_ng, beta, _, seed, box = gold["recipe"]
    print("N_g = 512 field: generating on the host", flush=True)
    delta = make_field(FieldRecipe(int(ng), box_len=float(box), n_s=float(n_s), f_ng=float(f_ng), beta=float(beta),
                                   seed=int(seed)))
    assert field_digest(delta) == str(gold["digest"]), "regenerated field differs from the stored one"
    return gold, delta


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [2], ids=["f64"])
def test_ng512_sampled_bins_against_stored_oracle(ng512_field, prec):
    """The N_g = 512 workload (60 k1 x 20 mu x 15 t, the bench configuration)
    against the float64 oracle on the 900 bins of its three lowest k1 shells,
    the ones the oracle can afford at this size (stored by make_golden.py
    with the oracle's bin filter).  The float64 path only: each plan at this
    size takes about a minute to build, and test_ng512 ties the float32 path
    to the float64 one on every bin."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_14513_amd import bk

    gold, delta = ng512_field
    ng, n_k1, k1_min, k1_max, n_mu, n_t, even, box = gold["binning"]
    bins = gold["sampled_bins"]
    print(f"N_g = 512 sampled-bin parity prec={prec}", flush=True)
    b = bk.make_binning(int(ng), int(n_k1), float(k1_min), float(k1_max), int(n_mu), int(n_t), box_len=float(box),
                        even_l_only=int(even))
    est = bk.Estimator(b, prec=prec)
    try:
        t = torch.from_numpy(delta.astype(np.float32) if prec == 1 else delta).cuda()
        s = torch.cuda.current_stream().cuda_stream
        est.load(t, s)
        est.estimate(s)
        B = est.multipoles()[0]
        counts = est.counts()
        lms = est.lm_list()
        del t
    finally:
        est.close()
    assert [tuple(x) for x in gold["lms"].tolist()] == lms
    assert np.array_equal(counts.ravel()[bins], gold["counts"].ravel()[bins])
    nlm = len(lms)
    Bs, Rs = B.reshape(nlm, -1)[:, bins], gold["B"].reshape(nlm, -1)[:, bins]
    assert np.array_equal(np.isnan(Bs), np.isnan(Rs))
    ok = ~np.isnan(Rs)
    assert ok.sum() > 100 * nlm // 2
    err = np.array([np.max(np.abs(Bs[j][ok[j]] - Rs[j][ok[j]])) / np.max(np.abs(Rs[j][ok[j]])) for j in range(nlm)])
    print(f"  max error per multipole over {ok[0].sum()} bins {err.max():.3e}", flush=True)
    assert err.max() < (1e-11 if prec == 2 else 1e-5), err
