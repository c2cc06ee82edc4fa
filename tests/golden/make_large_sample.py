"""Write tests/golden/large_oracle_sample.npz: the FP64 oracle's y = M x at a
sample of 64 spheres of the N = 100,000, phi = 0.4 workload (all spheres are
sources). Calls only oracle/ and the seeded input generators.

Oracle settings: xi = 0.1, both Gaussian tails cut at exp(-25) (tol_exp = 5),
which the converged-mode comparison puts at about 1e-10 relative.
Run: python tests/golden/make_large_sample.py   (a few minutes on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ewald  # noqa: E402
from paper_1506_08481_amd import workloads as wl  # noqa: E402

SEED_POS, SEED_X, NSAMPLE = 3000, 3001, 64


def main():
    s = wl.config_large(seed=SEED_POS)
    x = wl.force_moments(s.n, SEED_X)
    targets = np.sort(np.random.Generator(np.random.PCG64(77)).choice(s.n, NSAMPLE, replace=False))
    p = ewald.converged_params(s.box, s.radius, xi=0.1, tol_exp=5.0)
    t0 = time.time()
    y = ewald.apply(s.pos, s.radius, s.box, x, p, targets=targets)
    np.savez(os.path.join(HERE, "large_oracle_sample.npz"), targets=targets, y=y,
             pos_checksum=np.array([s.pos.sum(), (s.pos ** 2).sum()]),
             x_checksum=np.array([x.sum(), (x ** 2).sum()]))
    print(f"wrote {len(targets)} targets in {time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
