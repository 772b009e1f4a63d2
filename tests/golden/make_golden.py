"""Write oracle expected values for the full-size parity tests.

Calls only the oracle (float64, CPU) and the seeded input generator:
    python tests/golden/make_golden.py [name ...]
For each workload it stores, in tests/golden/oracle_<name>.npz: the multipoles
B [n_lm][n_k1][n_mu][n_t] (NaN where empty), the triangle counts, the (l, m)
list, the binning and recipe, and the SHA-256 of the generated field so a test
can confirm it regenerated the same input.
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.estimator import estimate_streaming_binnings  # noqa: E402
from oracle.geometry import Binning  # noqa: E402
from synth import FieldRecipe, field_digest, make_field  # noqa: E402

# Single-realisation workloads; field P ~ k^-2, f_NG = 0.5, beta = 0.5:
#   ng128, ng256  N_g = 128 (20 k1 x 10 mu x 10 t) and 256 (40 k1 x 20 mu x 10 t), seed 0
#   ng128_all_l   the N_g = 128 workload with every l <= 6 (odd l from the imaginary part)
#   ng96          the first N_g = 96 field of the uneven batch (seed 24; 20 k1 on [1, 32), 10 x 10)
#   ng192         N_g = 192, 20 k1 shells on [1, 64), 10 mu x 10 t, seed 0
#   val384        the validation setup of Sec. III.B-D: N_g = 384, L = 215 Mpc,
#                 k1 = 2.1 +- 0.1 Mpc^-1, 12 mu x 12 t, beta = 1, seed 1000
#   ng512_lowk    the N_g = 512 workload (60 k1 x 20 mu x 15 t, n_s = -1.5, seed 0),
#                 sampled: the 900 bins of its three lowest k1 shells only
KF_VAL = 2.0 * math.pi / 215.0  # fundamental mode of the validation box, Mpc^-1
CONFIGS = {
    "ng128": (Binning(128, 20, 1.0, 128 / 3, 10, 10), FieldRecipe(128, n_s=-2.0, f_ng=0.5, beta=0.5, seed=0)),
    "ng256": (Binning(256, 40, 1.0, 256 / 3, 20, 10), FieldRecipe(256, n_s=-2.0, f_ng=0.5, beta=0.5, seed=0)),
    "ng128_all_l": (Binning(128, 20, 1.0, 128 / 3, 10, 10, even_l_only=False),
                    FieldRecipe(128, n_s=-2.0, f_ng=0.5, beta=0.5, seed=0)),
    "ng96": (Binning(96, 20, 1.0, 32.0, 10, 10), FieldRecipe(96, n_s=-2.0, f_ng=0.5, beta=0.5, seed=24)),
    "ng192": (Binning(192, 20, 1.0, 64.0, 10, 10), FieldRecipe(192, n_s=-2.0, f_ng=0.5, beta=0.5, seed=0)),
    "val384": (Binning(384, 1, 2.0 / KF_VAL, 2.2 / KF_VAL, 12, 12, box_len=215.0),
               FieldRecipe(384, box_len=215.0, n_s=-2.0, f_ng=0.5, beta=1.0, seed=1000)),
    "ng512_lowk": (Binning(512, 60, 1.0, 512 / 3, 20, 15), FieldRecipe(512, n_s=-1.5, f_ng=0.5, beta=0.5, seed=0)),
}
# sampled workloads: number of lowest k1 shells computed
SAMPLED_SHELLS = {"ng512_lowk": 3}


def main(names):
    for name in names:
        b, rec = CONFIGS[name]
        t0 = time.time()
        delta = make_field(rec)
        workers = int(os.environ.get("ORACLE_WORKERS", "8"))
        extra = {}
        if name in SAMPLED_SHELLS:
            # only the combinations of the lowest shells; their sides all have k < the shells' top edge
            shells = SAMPLED_SHELLS[name]
            top = b.k1_min + shells * (b.k1_max - b.k1_min) / b.n_k1
            bins = np.arange(shells * b.n_mu * b.n_t)
            res = estimate_streaming_binnings(delta, [b], workers=min(workers, 4), chunks=4, bins=bins,
                                              plane_filter=lambda pt: max(abs(n) for n in pt) < top)[0]
            extra["sampled_bins"] = bins
        else:
            res = estimate_streaming_binnings(delta, [b], workers=workers, chunks=256)[0]
        out = os.path.join(HERE, f"oracle_{name}.npz")
        np.savez_compressed(
            out,
            **extra,
            B=res.B,
            counts=res.counts,
            lms=np.array(res.lms),
            binning=np.array([b.ng, b.n_k1, b.k1_min, b.k1_max, b.n_mu, b.n_t, int(b.even_l_only), b.length]),
            recipe=np.array([rec.ng, rec.n_s, rec.f_ng, rec.beta, rec.sigma_g, rec.seed, rec.length]),
            digest=np.array(field_digest(delta)),
        )
        print(f"{name}: wrote {out} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["ng128", "ng256"])
