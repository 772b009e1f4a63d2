"""The allocation-free estimate (bk_estimate_noalloc) against bk_estimate.

The entry point runs the plan's kernels on caller input and output buffers
with the library's static device scratch for the intermediate buffers; its
results must equal the allocating path's bit for bit (same kernels, same
order), on two calls in a row, the second with a smaller input, and the
oracle's to the parity bar.  A plan whose working set exceeds the scratch is
refused before anything is launched.
"""
import numpy as np
import pytest

from oracle.estimator import estimate
from oracle.geometry import Binning
from synth import FieldRecipe, make_field

pytestmark = pytest.mark.gpu

TOL = {2: 1e-11, 1: 1e-5}


def _lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_14513_amd import bk

    return torch, bk


def _run_both(torch, bk, plan, fields, prec):
    """(allocating path's B, allocation-free path's B) for the stacked fields."""
    s = torch.cuda.current_stream().cuda_stream
    t = torch.from_numpy(fields.astype(np.float32) if prec == 1 else fields).cuda()
    batch = fields.shape[0]
    bk.bk_load_grid(plan, t.data_ptr(), prec, batch, True, s)
    bk.bk_estimate(plan, s)
    ref = bk.bk_get_multipoles(plan, batch)
    n_lm, n_k1, n_mu, n_t = bk.bk_query_sizes(plan)
    out = torch.full((batch, n_lm, n_k1, n_mu, n_t), -1.0, dtype=torch.float64, device="cuda")
    bk.bk_estimate_noalloc(plan, t.data_ptr(), prec, batch, out.data_ptr(), s)
    torch.cuda.synchronize()
    return ref, out.cpu().numpy()


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_noalloc_matches_allocating_path(prec):
    torch, bk = _lib()
    big = (48, 4, 2.0, 16.0, 6, 5)
    small = (32, 4, 1.0, 32 / 3, 5, 4)
    fb = np.stack([make_field(FieldRecipe(48, n_s=-1.5, f_ng=0.5, beta=1.0, seed=s)) for s in (2, 3)])
    fs = make_field(FieldRecipe(32, n_s=-2.0, f_ng=0.5, beta=0.5, seed=1))[None]
    p_big = bk.bk_plan_create(bk.make_binning(*big), prec, 0, 2)
    p_small = bk.bk_plan_create(bk.make_binning(*small), prec, 0, 1)
    try:
        # first call: two N_g = 48 fields; second: one N_g = 32 field, then one N_g = 48 field
        for plan, fields, args in ((p_big, fb, big), (p_small, fs, small), (p_big, fb[1:], big)):
            ref, got = _run_both(torch, bk, plan, fields, prec)
            assert np.array_equal(np.isnan(ref), np.isnan(got))
            ok = ~np.isnan(ref)
            assert np.array_equal(ref[ok], got[ok])
            oracle = estimate(fields[0], Binning(*args))
            B = got[0].reshape(oracle.B.shape[0], -1)
            R = oracle.B.reshape(oracle.B.shape[0], -1)
            okr = ~np.isnan(R)
            for j in range(R.shape[0]):
                assert np.max(np.abs(B[j][okr[j]] - R[j][okr[j]])) < TOL[prec] * np.max(np.abs(R[j][okr[j]]))
    finally:
        bk.bk_plan_destroy(p_big)
        bk.bk_plan_destroy(p_small)


def test_noalloc_refuses_plans_beyond_the_scratch():
    torch, bk = _lib()
    plan = bk.bk_plan_create(bk.make_binning(96, 20, 1.0, 32.0, 10, 10), bk.BK_F32, 0, 1)
    try:
        t = torch.zeros((1, 96, 96, 96), dtype=torch.float32, device="cuda")
        out = torch.zeros(16 * 2000, dtype=torch.float64, device="cuda")
        with pytest.raises(bk.BkError) as e:
            bk.bk_estimate_noalloc(plan, t.data_ptr(), bk.BK_F32, 1, out.data_ptr(), 0)
        assert e.value.status == bk.BK_ERR_SIZE
        assert "scratch" in str(e.value)
        assert torch.count_nonzero(out).item() == 0
    finally:
        bk.bk_plan_destroy(plan)
