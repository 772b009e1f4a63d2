"""The stored oracle values under tests/golden are what the committed oracle
computes: for each stored workload small enough for the CPU suite, the
field regenerates to the stored digest, and the oracle rerun on the bins of
its two lowest k1 shells (restricted to the plane triples that reach them)
reproduces the stored multipoles to rounding and the triangle counts
exactly."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

from make_golden import CONFIGS  # noqa: E402

from oracle.estimator import estimate_streaming_binnings  # noqa: E402
from synth import field_digest, make_field  # noqa: E402


@pytest.mark.parametrize("name", ["ng96", "ng128", "ng128_all_l", "ng192", "ng256"])
def test_stored_oracle_values_are_reproduced(name):
    b, rec = CONFIGS[name]
    delta = make_field(rec)
    g = np.load(os.path.join(HERE, "golden", f"oracle_{name}.npz"))
    assert str(g["digest"]) == field_digest(delta)
    shells = 2
    top = b.k1_min + shells * (b.k1_max - b.k1_min) / b.n_k1
    bins = np.arange(shells * b.n_mu * b.n_t)
    res = estimate_streaming_binnings(delta, [b], workers=1, chunks=4, bins=bins,
                                      plane_filter=lambda pt: max(abs(n) for n in pt) < top)[0]
    n_lm = len(res.lms)
    assert [tuple(x) for x in g["lms"]] == [tuple(x) for x in res.lms]
    B = res.B.reshape(n_lm, -1)[:, bins]
    ref = g["B"].reshape(n_lm, -1)[:, bins]
    ok = ~np.isnan(ref)
    assert np.array_equal(np.isnan(B), ~ok)
    assert ok.any()
    assert np.max(np.abs(B[ok] - ref[ok])) <= 1e-13 * np.nanmax(np.abs(g["B"]))
    assert np.array_equal(res.counts.reshape(-1)[bins], g["counts"].reshape(-1)[bins])
