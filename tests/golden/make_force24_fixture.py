"""Write tests/golden/force24_oracle_sample.npz: the oracle's fermion force
(gradient of S = phi^dag (D^dag D)^{-1} phi with respect to the fat and Naik
links) on the 24^4 HISQ-style workload (eps 0.5, m = 0.01, one Gaussian phi,
the seeds of the force benchmark), at 256 seeded fat-link and 256 seeded
Naik-link positions, plus S.  Calls only oracle/ and the input generators
(about an hour of one CPU core: two FP64 Schur CG solves in numpy).

    python tests/golden/make_force24_fixture.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import solvers as sol  # noqa: E402
from paper_2212_12559_amd import latgen  # noqa: E402

DIMS = (24, 24, 24, 24)
EPS, SEED, MASS = 0.5, 20221228, 0.01
C1, C3 = 9.0 / 8.0, -1.0 / 24.0
NSAMPLE = 256
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "force24_oracle_sample.npz")


def sample_positions():
    """(mu, t, z, y, x) of the sampled links, fat then Naik (seeded)."""
    rng = np.random.default_rng(24242424)
    X, Y, Z, T = DIMS
    hi = np.array([4, T, Z, Y, X])
    return rng.integers(0, hi, size=(NSAMPLE, 5)), rng.integers(0, hi, size=(NSAMPLE, 5))


def main():
    t0 = time.time()
    W, N, rng = latgen.hisq_style_links(DIMS, EPS, SEED)
    phi = latgen.fine_vectors(DIMS, 1, rng)[0]
    S, gW, gN, _, _ = sol.force(W, N, MASS, C1, C3, phi, tol=1e-11)
    pw, pn = sample_positions()
    sw = np.stack([gW[tuple(p)] for p in pw])
    sn = np.stack([gN[tuple(p)] for p in pn])
    np.savez(OUT, S=S, pos_fat=pw, pos_naik=pn, grad_fat=sw, grad_naik=sn,
             max_abs_fat=np.max(np.abs(gW)), max_abs_naik=np.max(np.abs(gN)))
    print(f"S = {S!r}, wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
