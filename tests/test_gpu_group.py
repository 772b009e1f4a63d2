"""Plan groups: several plans (different N_g, batched fields) captured into one
hipGraph and replayed.  Every replay, with eager work and synchronisations in
between, must reproduce the eager per-plan results bit for bit; the eager
results themselves are checked against the oracle."""
import numpy as np
import pytest

from oracle.estimator import estimate
from oracle.geometry import Binning
from synth import FieldRecipe, make_field

pytestmark = pytest.mark.gpu

SPECS = [  # (binning args, seeds)
    ((16, 3, 2.0, 5.0, 5, 3), (0, 1)),
    ((24, 3, 1.0, 8.0, 4, 4), (2,)),
    ((32, 4, 1.0, 32 / 3, 5, 4), (3, 4, 5)),
]


@pytest.mark.parametrize("prec", [1, 2], ids=["f32", "f64"])
def test_group_graph_replays_match_eager(prec):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_14513_amd import bk

    stream = torch.cuda.current_stream().cuda_stream
    plans, fields, eager = [], [], []
    try:
        for args, seeds in SPECS:
            f = np.stack([make_field(FieldRecipe(args[0], seed=s)) for s in seeds])
            t = torch.from_numpy(f).cuda()
            plan = bk.bk_plan_create(bk.make_binning(*args), prec, 0, len(seeds))
            plans.append(plan)
            fields.append((t, f))
            bk.bk_load_grid(plan, t.data_ptr(), bk.BK_F64, len(seeds), True, stream)
            bk.bk_estimate(plan, stream)
            eager.append(bk.bk_get_multipoles(plan, len(seeds)))
        # eager results against the oracle
        tol = 1e-11 if prec == 2 else 1e-5
        for (args, seeds), (_, f), B in zip(SPECS, fields, eager):
            for i in range(len(seeds)):
                ref = estimate(f[i], Binning(*args)).B
                ok = ~np.isnan(ref)
                assert np.array_equal(np.isnan(B[i]), ~ok)
                assert np.max(np.abs(B[i][ok] - ref[ok])) < tol * np.max(np.abs(ref[ok]))
        group = bk.bk_group_create(plans)
        try:
            for rep in range(3):
                bk.bk_group_estimate(group, stream)
                torch.cuda.synchronize()
                for (args, seeds), plan, B in zip(SPECS, plans, eager):
                    G = bk.bk_get_multipoles(plan, len(seeds))
                    assert np.array_equal(np.isnan(G), np.isnan(B))
                    ok = ~np.isnan(B)
                    assert np.array_equal(G[ok], B[ok]), f"replay {rep} differs"
                # eager work on the same stream between replays
                x = torch.randn(1 << 20, device="cuda")
                (x * 2).sum().item()
                bk.bk_estimate(plans[0], stream)
                torch.cuda.synchronize()
            # a different batch size in one member forces a new capture
            t0 = fields[2][0][:1].contiguous()
            bk.bk_load_grid(plans[2], t0.data_ptr(), bk.BK_F64, 1, True, stream)
            bk.bk_group_estimate(group, stream)
            G = bk.bk_get_multipoles(plans[2], 1)
            ok = ~np.isnan(eager[2][0])
            assert np.array_equal(G[0][ok], eager[2][0][ok])
        finally:
            bk.bk_group_destroy(group)
    finally:
        for p in plans:
            bk.bk_plan_destroy(p)


def test_group_errors():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_14513_amd import bk

    plan = bk.bk_plan_create(bk.make_binning(16, 3, 2.0, 5.0, 5, 3), bk.BK_F64, 0, 1)
    try:
        with pytest.raises(bk.BkError) as e:
            bk.bk_group_create([plan, plan])
        assert e.value.status == bk.BK_ERR_ARG
        group = bk.bk_group_create([plan])
        try:
            with pytest.raises(bk.BkError) as e:
                bk.bk_group_estimate(group, 0)  # nothing loaded yet
            assert e.value.status == bk.BK_ERR_STATE
        finally:
            bk.bk_group_destroy(group)
    finally:
        bk.bk_plan_destroy(plan)
