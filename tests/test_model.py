"""The library's analytic predictions (host-only C ABI) against the oracle.

bk_discrete_prediction is [B_l^m]_d of Sec. III.C (Eq. 17 at each kept
combination's mean sides, binned with Eq. 13's weights); bk_continuum_multipoles
is Eq. 4 by exact quadrature.  Both are independent C++ restatements; the
oracle's numpy versions (oracle/analytic.py) are the references, themselves
pinned in test_oracle_pins.py.
"""
import numpy as np
import pytest

from oracle.analytic import continuum_multipole, discrete_prediction
from oracle.geometry import Binning, make_geometry
from paper_2405_14513_amd import bk


@pytest.mark.parametrize(
    "args, model",
    [
        ((24, 3, 1.0, 8.0, 4, 4, 37.5), (2.0, -2.0, 0.5, 1.0)),
        ((32, 4, 1.0, 32 / 3, 5, 4, 0.0), (0.7, -1.5, 0.5, 0.5)),
        ((16, 3, 2.0, 5.0, 5, 3, 0.0), (1.3, -2.0, 0.25, 0.0)),
    ],
)
@pytest.mark.parametrize("even", [True, False], ids=["even_l", "all_l"])
def test_discrete_prediction_matches_oracle(args, model, even):
    ng, n_k1, k1_min, k1_max, n_mu, n_t, box = args
    b = Binning(ng, n_k1, k1_min, k1_max, n_mu, n_t, box_len=box if box > 0 else None, even_l_only=even)
    ref = discrete_prediction(make_geometry(b), *model)
    got = bk.bk_discrete_prediction(bk.make_binning(ng, n_k1, k1_min, k1_max, n_mu, n_t, box_len=box,
                                                    even_l_only=int(even)), *model)
    assert got.shape == ref.shape
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    for j in range(ref.shape[0]):
        scale = np.abs(ref[j][ok[j]]).max()
        assert np.abs(got[j][ok[j]] - ref[j][ok[j]]).max() <= 1e-12 * scale, j


@pytest.mark.parametrize("mu, t, beta", [(0.6, 0.9, 1.0), (0.8, 0.8, 0.5), (0.95, 0.7, 1.0), (1.0, 0.5, 0.3)])
def test_continuum_multipoles_match_oracle(mu, t, beta):
    got = bk.bk_continuum_multipoles(6, 6, mu, t, beta)
    lms = [(l, m) for l in range(0, 7, 2) for m in range(0, l + 1)]
    ref = np.array([continuum_multipole(l, m, mu, t, beta).real for l, m in lms])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_continuum_b00_without_rsd_is_one():
    """beta = 0: the angular factor is 1, so [B_0^0]_c / B_r = 1 and the rest vanish."""
    got = bk.bk_continuum_multipoles(6, 6, 0.7, 0.8, 0.0)
    assert abs(got[0] - 1.0) < 1e-14
    assert np.abs(got[1:]).max() < 1e-14


def test_prediction_errors():
    with pytest.raises(bk.BkError) as e:
        bk.bk_discrete_prediction(bk.make_binning(20, 3, 2.0, 5.0, 5, 3), 1.0, -2.0, 0.5, 1.0)
    assert e.value.status == bk.BK_ERR_ARG
    with pytest.raises(bk.BkError) as e:
        bk.bk_discrete_prediction(bk.make_binning(16, 3, 2.0, 5.0, 5, 3), float("nan"), -2.0, 0.5, 1.0)
    assert e.value.status == bk.BK_ERR_ARG
    with pytest.raises(bk.BkError) as e:
        bk.bk_continuum_multipoles(6, 7, 0.5, 0.5, 1.0)
    assert e.value.status == bk.BK_ERR_ARG
    with pytest.raises(bk.BkError) as e:
        bk.bk_continuum_multipoles(6, 6, 1.0, 1.0, 1.0)  # k3 = 0
    assert e.value.status == bk.BK_ERR_ARG


def test_prediction_matches_validation_golden():
    """The N_g = 384 validation setup: the library's [B]_d equals the stored
    oracle values (tests/golden/validation_ng384.npz) for all three binnings."""
    import os

    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "validation_ng384.npz"))
    k1_min, k1_max = g["k1"]
    for n in (12, 8, 6):
        got = bk.bk_discrete_prediction(bk.make_binning(384, 1, k1_min, k1_max, n, n, box_len=215.0),
                                        float(g["amp"]), -2.0, 0.5, 1.0)
        ref = g[f"Bd_{n}"]
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        ok = ~np.isnan(ref)
        for j in range(ref.shape[0]):
            assert np.abs(got[j][ok[j]] - ref[j][ok[j]]).max() <= 1e-11 * np.abs(ref[j][ok[j]]).max(), (n, j)


def test_mean_value_prediction_tracks_the_exact_first_order_expectation():
    """At the validation setup, the paper's [B]_d (B_s at each combination's
    mean sides) against the estimator's exact first-order expectation Bexact
    (Eq. 13 over every triangle's own B_s; both stored by make_validation.py
    from the oracle): the monopole differs by well under a percent in the
    median and by at most a few percent in any bin, so [B]_d is an adequate
    reference at the ensemble's noise level."""
    import os

    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "validation_ng384.npz"))
    for n in (12, 8, 6):
        bd, bx = g[f"Bd_{n}"][0], g[f"Bexact_{n}"][0]
        ok = ~np.isnan(bd)
        assert np.array_equal(ok, ~np.isnan(bx))
        rel = bx[ok] / bd[ok] - 1.0
        assert abs(np.median(rel)) < 0.01, n
        assert np.abs(rel).max() < 0.05, n
