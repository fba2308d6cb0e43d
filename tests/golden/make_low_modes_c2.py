"""Writes low_modes_8x8x8x16.json: the 13 eigenvalues of smallest |lambda| of K on the 8^3x16
workload's stout-smeared links (the 12 deflated modes and the first undeflated one), from the
oracle's ARPACK implicitly restarted Lanczos on a Chebyshev filter of K^2 followed by Rayleigh-Ritz
with K (oracle.eigen.low_modes), with their residuals.  Inputs come from latgen by the stored seed;
only oracle/ computes.

Run once (a few minutes):  python tests/golden/make_low_modes_c2.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import latgen  # noqa: E402
from oracle.eigen import low_modes  # noqa: E402

DIMS = (8, 8, 8, 16)
N_EV, LMAX = 13, 6.5
SEED = latgen.seed_for("gauge", 2)


def main():
    t0 = time.time()
    u = latgen.smeared_field(DIMS, SEED)
    lam, phi, res = low_modes(u, N_EV, LMAX, filter_degree=24, tol=1e-11)
    out = {"what": "eigenvalues of K = gamma5 (D_W - 1.5) with the smallest |lambda| (ascending "
                   "|lambda|), oracle.eigen.low_modes (ARPACK on a Chebyshev filter of K^2, then "
                   "Rayleigh-Ritz with K)",
           "dims": list(DIMS), "lmax": LMAX, "gauge_seed": SEED,
           "links": "latgen.smeared_field(dims, gauge_seed): noise 0.3, 3 stout steps rho 0.1",
           "lambda": [float(x) for x in lam], "residuals": [float(x) for x in res],
           "seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "low_modes_8x8x8x16.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["lambda"]), flush=True)


if __name__ == "__main__":
    main()
