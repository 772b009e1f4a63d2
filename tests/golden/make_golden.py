"""Write oracle expected values for the full-size parity tests.

Calls only the oracle (float64, CPU) and the seeded input generator:
    python tests/golden/make_golden.py [ng ...]
For each grid it stores, in tests/golden/oracle_ng<N>.npz: the multipoles
B [n_lm][n_k1][n_mu][n_t] (NaN where empty), the triangle counts, the (l, m)
list, the binning and recipe, and the SHA-256 of the generated field so a test
can confirm it regenerated the same input.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.estimator import estimate_streaming  # noqa: E402
from oracle.geometry import Binning  # noqa: E402
from synth import FieldRecipe, field_digest, make_field  # noqa: E402

# The two single-realisation workloads: N_g = 128 (20 k1 x 10 mu x 10 t) and
# N_g = 256 (40 k1 x 20 mu x 10 t); field: P ~ k^-2, f_NG = 0.5, beta = 0.5, seed 0.
CONFIGS = {
    128: (Binning(128, 20, 1.0, 128 / 3, 10, 10), FieldRecipe(128, n_s=-2.0, f_ng=0.5, beta=0.5, seed=0)),
    256: (Binning(256, 40, 1.0, 256 / 3, 20, 10), FieldRecipe(256, n_s=-2.0, f_ng=0.5, beta=0.5, seed=0)),
}


def main(ngs):
    for ng in ngs:
        b, rec = CONFIGS[ng]
        t0 = time.time()
        delta = make_field(rec)
        res = estimate_streaming(delta, b, workers=int(os.environ.get("ORACLE_WORKERS", "8")), chunks=256)
        out = os.path.join(HERE, f"oracle_ng{ng}.npz")
        np.savez_compressed(
            out,
            B=res.B,
            counts=res.counts,
            lms=np.array(res.lms),
            binning=np.array([b.ng, b.n_k1, b.k1_min, b.k1_max, b.n_mu, b.n_t]),
            recipe=np.array([rec.ng, rec.n_s, rec.f_ng, rec.beta, rec.sigma_g, rec.seed]),
            digest=np.array(field_digest(delta)),
        )
        print(f"ng={ng}: wrote {out} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [128, 256])
