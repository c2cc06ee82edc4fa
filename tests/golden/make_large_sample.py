"""Write the FP64 oracle's y = M x at a sample of 64 spheres of two large
workloads (all spheres are sources). Calls only oracle/ and the seeded input
generators.

  tests/golden/large_oracle_sample.npz       N = 100,000 equal spheres, phi = 0.4
  tests/golden/bidisperse_oracle_sample.npz  N = 40,000 spheres of radii 1 and 2
                                             (equal volume per species), phi = 0.35

Oracle settings: both Gaussian tails cut at exp(-25) (tol_exp = 5), which the
converged-mode comparison puts at about 1e-10 relative; xi = 0.1 for the
first workload and 0.12 for the second, whose smaller box (L = 94.7) would
otherwise put r_c = tol_exp / xi above L/2 (the converged result does not
depend on xi; below L/2 the oracle's real-space sum runs in chunks).
Run: python tests/golden/make_large_sample.py [large|bidisperse]
(a few minutes each on 8 cores)
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
BI_N, BI_PHI, BI_SEED_POS, BI_SEED_X = 40000, 0.35, 4000, 4001


def bidisperse_workload():
    """The bidisperse suspension of bidisperse_oracle_sample.npz."""
    return wl.bidisperse(BI_N, BI_PHI, BI_SEED_POS, a1=1.0, a2=2.0)


def write(name, s, x, xi):
    targets = np.sort(np.random.Generator(np.random.PCG64(77)).choice(s.n, NSAMPLE, replace=False))
    p = ewald.converged_params(s.box, s.radius, xi=xi, tol_exp=5.0)
    t0 = time.time()
    y = ewald.apply(s.pos, s.radius, s.box, x, p, targets=targets)
    np.savez(os.path.join(HERE, name), targets=targets, y=y,
             pos_checksum=np.array([s.pos.sum(), (s.pos ** 2).sum()]),
             x_checksum=np.array([x.sum(), (x ** 2).sum()]))
    print(f"{name}: wrote {len(targets)} targets in {time.time() - t0:.0f}s")


def main():
    which = sys.argv[1:] or ["large", "bidisperse"]
    if "large" in which:
        s = wl.config_large(seed=SEED_POS)
        write("large_oracle_sample.npz", s, wl.force_moments(s.n, SEED_X), 0.1)
    if "bidisperse" in which:
        s = bidisperse_workload()
        write("bidisperse_oracle_sample.npz", s, wl.force_moments(s.n, BI_SEED_X), 0.12)


if __name__ == "__main__":
    main()
