"""Writes force_directional_24x24x24x48.json: oracle values of the force workload's derivative
along seeded directions, for the full-size parity check of the device force (degree 299 on a
24^3x48 lattice, where the oracle's reverse sweep would need N stored FP64 vectors).

For L(U) = Re<chi, p(K/lmax) psi> and a direction Y (complex Gaussian on every link component),
dL/d eps of L(U + eps Y) is computed by ``oracle.force.sign_force_directional`` (forward mode,
four live vectors) on the exact FP64 inputs and on the same inputs rounded to FP32.  The device
force G satisfies Re sum tr(G^+ Y) = dL/d eps, so each stored value checks G along Y.  Inputs
come from ``latgen`` by the seeds stored in the file; only ``oracle/`` computes.

Run once (about 40 minutes on four cores):  python tests/golden/make_force_directional.py
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import latgen  # noqa: E402
from oracle import chebyshev as och  # noqa: E402
from oracle import force as oforce  # noqa: E402

DIMS = (24, 24, 24, 48)
DEGREE, EPS, LMAX = 300, 0.05, 6.5
SEEDS = {"gauge": latgen.seed_for("gauge", 5), "psi": latgen.seed_for("spinor", 5),
         "chi": latgen.seed_for("spinor", 5, 1)}
DIRECTION_SEEDS = [latgen.seed_for("direction", 0, 50), latgen.seed_for("direction", 0, 51)]
OUT = os.path.join(HERE, "force_directional_24x24x24x48.json")

_inputs = {}


def direction(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def work(job):
    kind, k = job
    u, chi, psi = _inputs[kind]
    y = direction(u.shape, DIRECTION_SEEDS[k])
    alpha = och.coeffs_sign_interp(DEGREE, EPS)
    t0 = time.time()
    v = oforce.sign_force_directional(u, chi, psi, alpha, LMAX, y)
    return kind, k, v, time.time() - t0


def main():
    t0 = time.time()
    u = latgen.smeared_field(DIMS, SEEDS["gauge"])
    psi = latgen.gaussian_spinor(DIMS, SEEDS["psi"])
    chi = latgen.gaussian_spinor(DIMS, SEEDS["chi"])
    _inputs["exact"] = (u, chi, psi)
    _inputs["f32_rounded"] = (latgen.round_to_f32(u), latgen.round_to_f32(chi),
                              latgen.round_to_f32(psi))
    print(f"inputs {time.time() - t0:.0f} s", flush=True)
    jobs = [(kind, k) for kind in ("exact", "f32_rounded") for k in range(len(DIRECTION_SEEDS))]
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        res = pool.map(work, jobs)
    out = {"what": "dL/d eps of L(U + eps Y) = Re<chi, p(K/lmax) psi>, forward mode through the "
                   "forward Chebyshev recurrence (oracle.force.sign_force_directional)",
           "dims": list(DIMS), "degree": DEGREE, "eps": EPS, "lmax": LMAX, "m_w": 1.5,
           "coefficients": "oracle.chebyshev.coeffs_sign_interp(degree, eps)",
           "links": "latgen.smeared_field(dims, gauge seed): noise 0.3, 3 stout steps rho 0.1",
           "seeds": SEEDS, "direction_seeds": DIRECTION_SEEDS,
           "direction": "complex Gaussian a + ib on every link component (a, b ~ N(0, 1), "
                        "PCG64(seed), array shape of U)",
           "values": {kind: [None] * len(DIRECTION_SEEDS) for kind in ("exact", "f32_rounded")},
           "seconds": {}}
    for kind, k, v, sec in res:
        out["values"][kind][k] = v
        out["seconds"][f"{kind}_{k}"] = round(sec, 1)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["values"]), flush=True)


if __name__ == "__main__":
    main()
