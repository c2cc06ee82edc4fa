"""Write the FP64 oracle's y = M x at sampled spheres of two large workloads
(every sphere is a source; the oracle evaluates the sum only at the sampled
targets). Calls only oracle/ and the seeded input generators.

  tests/golden/large_oracle_sample.npz       N = 100,000 equal spheres, phi = 0.4,
                                             2,000 targets drawn uniformly
  tests/golden/bidisperse_oracle_sample.npz  N = 40,000 spheres of radii 1 and 2
                                             (equal volume per species), phi = 0.35,
                                             64 targets

Oracle settings: both Gaussian tails cut at exp(-25) (tol_exp = 5), which the
converged-mode comparison puts at about 1e-10 relative. The converged result
does not depend on xi, so xi only balances the oracle's own cost: its
real-space sum grows as (targets)/xi^3 and its structure sums as N xi^3.
The 2,000 targets of the first workload are split over worker processes,
each of which evaluates the oracle at its share of the targets (xi = 0.2
balances the two parts per worker; each worker peaks near 10 GB, so three
run at once on a 64 GB machine); the second workload uses xi = 0.12, which
keeps r_c = tol_exp / xi below L/2 (L = 94.7).
Run: python tests/golden/make_large_sample.py [large|bidisperse]
(about 30 minutes for the first on 3 worker processes, 90 s for the second)
"""
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ewald  # noqa: E402
from paper_1506_08481_amd import workloads as wl  # noqa: E402

SEED_POS, SEED_X, NSAMPLE = 3000, 3001, 2000
XI_LARGE, WORKERS = 0.2, 3
BI_N, BI_PHI, BI_SEED_POS, BI_SEED_X, BI_NSAMPLE = 40000, 0.35, 4000, 4001, 64


def bidisperse_workload():
    """The bidisperse suspension of bidisperse_oracle_sample.npz."""
    return wl.bidisperse(BI_N, BI_PHI, BI_SEED_POS, a1=1.0, a2=2.0)


def sample_targets(n, count):
    return np.sort(np.random.Generator(np.random.PCG64(77)).choice(n, count, replace=False))


def _large_chunk(targets):
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)   # one BLAS thread per worker process
    s = wl.config_large(seed=SEED_POS)
    x = wl.force_moments(s.n, SEED_X)
    p = ewald.converged_params(s.box, s.radius, xi=XI_LARGE, tol_exp=5.0)
    return ewald.apply(s.pos, s.radius, s.box, x, p, targets=targets)


def save(name, s, x, targets, y, xi):
    np.savez(os.path.join(HERE, name), targets=targets, y=y,
             pos_checksum=np.array([s.pos.sum(), (s.pos ** 2).sum()]),
             x_checksum=np.array([x.sum(), (x ** 2).sum()]), xi=np.array(xi))


def main():
    which = sys.argv[1:] or ["large", "bidisperse"]
    if "large" in which:
        t0 = time.time()
        s = wl.config_large(seed=SEED_POS)
        x = wl.force_moments(s.n, SEED_X)
        targets = sample_targets(s.n, NSAMPLE)
        chunks = np.array_split(targets, WORKERS)
        with mp.get_context("spawn").Pool(WORKERS) as pool:
            ys = pool.map(_large_chunk, chunks)
        save("large_oracle_sample.npz", s, x, targets, np.concatenate(ys), XI_LARGE)
        print(f"large_oracle_sample.npz: {len(targets)} targets in {time.time() - t0:.0f}s", flush=True)
    if "bidisperse" in which:
        t0 = time.time()
        s = bidisperse_workload()
        x = wl.force_moments(s.n, BI_SEED_X)
        targets = sample_targets(s.n, BI_NSAMPLE)
        p = ewald.converged_params(s.box, s.radius, xi=0.12, tol_exp=5.0)
        y = ewald.apply(s.pos, s.radius, s.box, x, p, targets=targets)
        save("bidisperse_oracle_sample.npz", s, x, targets, y, 0.12)
        print(f"bidisperse_oracle_sample.npz: {len(targets)} targets in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
