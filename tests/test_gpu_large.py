"""Parity at the full benchmark size: N = 100,000 spheres at phi = 0.4,
grid 256^3, in the launch configurations the benchmark times, checked at
2,000 sampled spheres against the FP64 oracle
(tests/golden/large_oracle_sample.npz, written by
tests/golden/make_large_sample.py from the oracle alone): every FP32
configuration the benchmark may time holds the 1e-6 target there. A second
sample (bidisperse_oracle_sample.npz) covers a large suspension of two sphere
sizes, whose uneven neighbour lists take the wavefront-per-sphere pair sum."""
import math
import os

import numpy as np
import pytest

from paper_1506_08481_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "large_oracle_sample.npz")
GOLD_BI = os.path.join(HERE, "golden", "bidisperse_oracle_sample.npz")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def large():
    import torch
    d = np.load(GOLD)
    s = wl.config_large(seed=3000)
    x = wl.force_moments(s.n, 3001)
    # the stored sample belongs to exactly these inputs
    np.testing.assert_allclose([s.pos.sum(), (s.pos ** 2).sum()], d["pos_checksum"], rtol=1e-12)
    np.testing.assert_allclose([x.sum(), (x ** 2).sum()], d["x_checksum"], rtol=1e-12)
    dev = torch.device("cuda:0")
    return s, [torch.as_tensor(a, device=dev) for a in (s.pos, s.radius, x)], d["targets"], d["y"]


def _sample_error(cfg, precision, large):
    from paper_1506_08481_amd import seasd
    s, (P_, R_, X_), tg, yo = large
    xi, rcf, P, mf = cfg
    eng = seasd.Seasd(0, grid=256, P=P, m=mf * math.sqrt(math.pi * P), xi=xi, rc_factor=rcf,
                      precision=precision, checks=1)
    y = eng.apply(P_, R_, s.box, X_).cpu().numpy()
    eng.close()
    assert np.all(np.isfinite(y))
    return float(np.linalg.norm(y[tg] - yo) / np.linalg.norm(yo)), y


BLOCKS = {"U": slice(0, 3), "W": slice(3, 6), "E": slice(6, 11), "e": slice(11, 12)}


def _einf_blocks(y, yo):
    """eq. err-E per block over the sampled spheres."""
    out = {}
    for k, sl in BLOCKS.items():
        out[k] = float(np.max(np.linalg.norm(y[:, sl] - yo[:, sl], axis=1) / np.linalg.norm(yo[:, sl], axis=1)))
    return out


def test_large_fp64_reference(large):
    """The FP64 product that the benchmark measures its error against:
    Spectral Ewald error about 1e-8 at P = 18."""
    import bench
    from paper_1506_08481_amd import seasd
    err, _ = _sample_error(bench.REF, seasd.SEASD_FP64, large)
    print(f"fp64 ref sample error {err:.3e}")
    assert err < 5e-8


@pytest.mark.parametrize("k", [0, 1, 2])
def test_large_fp32_candidates(large, k):
    """Each FP32 configuration the benchmark may time holds the 1e-6 target
    on the 2,000-sphere sample; the per-block e_inf of eq. err-E is reported."""
    import bench
    from paper_1506_08481_amd import seasd
    err, y = _sample_error(bench.CANDIDATES[k], seasd.SEASD_FP32, large)
    tg, yo = large[2], large[3]
    print(f"fp32 candidate {bench.CANDIDATES[k]} sample error {err:.3e} over {len(tg)} spheres, "
          f"per-block e_inf {_einf_blocks(y[tg], yo)}")
    assert len(tg) >= 2000
    assert err <= 1e-6


@pytest.fixture(scope="module")
def bidisperse():
    import sys
    import torch
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_large_sample as mk
    d = np.load(GOLD_BI)
    s = mk.bidisperse_workload()
    x = wl.force_moments(s.n, mk.BI_SEED_X)
    np.testing.assert_allclose([s.pos.sum(), (s.pos ** 2).sum()], d["pos_checksum"], rtol=1e-12)
    np.testing.assert_allclose([x.sum(), (x ** 2).sum()], d["x_checksum"], rtol=1e-12)
    dev = torch.device("cuda:0")
    return s, [torch.as_tensor(a, device=dev) for a in (s.pos, s.radius, x)], d["targets"], d["y"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_large_bidisperse_autotuned(bidisperse, prec):
    """N = 40,000 spheres of radii 1 and 2 at phi = 0.35 in the configuration
    the autotuner picks for a 1e-6 target (128^3, r_c about 6 (a_i + a_j)): a
    large sphere then has about five times the mean number of neighbours, so
    once the first product has measured the lists, the pair sum runs with a
    wavefront per sphere. Both products agree to rounding; the second one's
    sample error is within twice the target."""
    from paper_1506_08481_amd import seasd
    s, (P_, R_, X_), tg, yo = bidisperse
    precision = seasd.SEASD_FP64 if prec == "fp64" else seasd.SEASD_FP32
    c = seasd.seasd_autotune(s.n, s.box, float(np.quantile(s.radius, 0.1)), float(s.radius.max()), 1e-6, precision)
    cfg = {k: v for k, v in c.as_dict().items() if k in ("grid", "P", "m", "xi", "rc_factor")}
    eng = seasd.Seasd(0, **cfg, precision=precision, checks=1)
    y1 = eng.apply(P_, R_, s.box, X_).cpu().numpy()   # one thread per sphere, lists measured
    y = eng.apply(P_, R_, s.box, X_).cpu().numpy()    # a wavefront per sphere
    eng.close()
    assert np.all(np.isfinite(y))
    assert np.linalg.norm(y - y1) <= 1e-12 * np.linalg.norm(y)
    err = float(np.linalg.norm(y[tg] - yo) / np.linalg.norm(yo))
    print(f"bidisperse {prec} {cfg} sample error {err:.3e}")
    assert err < 2e-6
