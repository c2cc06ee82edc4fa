"""Batched products: many suspensions of uneven size in one hipGraph launch.

* The plan's result equals the single-suspension product with the same
  configuration (same kernel bodies, same binned order) up to the order of
  the FP64 pair-sum additions.
* Replays of the captured graph, with eager work and synchronisation between
  them, each equal the single-suspension result for their own input.
* The autotuned FP32 configuration of a lognormal suspension meets 2e-6
  against the FP64 oracle.
* Members of the many-suspension workload match the FP64 oracle inside the
  batched plan.
"""
import math

import numpy as np
import pytest

from oracle import ewald
from paper_1506_08481_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_08481_amd import seasd
    return seasd


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


@pytest.fixture(scope="module")
def systems():
    specs = [(40, 0.1), (120, 0.45), (300, 0.3), (77, 0.2), (500, 0.4), (201, 0.15)]
    sus = [wl.lognormal(n, phi, 900 + k) for k, (n, phi) in enumerate(specs)]
    offs = np.concatenate([[0], np.cumsum([s.n for s in sus])])
    pos = np.concatenate([s.pos for s in sus])
    rad = np.concatenate([s.radius for s in sus])
    return sus, offs, pos, rad


def _individual(lib, s, cfg, x):
    eng = lib.Seasd(0)
    eng.config = cfg
    eng.set_config()
    y = eng.apply(_t(s.pos), _t(s.radius), s.box, _t(x))
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    eng.close()
    return out


def test_batch_equals_single_products_and_replays(lib, systems):
    sus, offs, pos, rad = systems
    eng = lib.Seasd(0, precision=lib.SEASD_FP32)
    plan = lib.Batch(eng, offs, _t(pos), _t(rad), [s.box for s in sus], target=1e-6)
    cfgs = plan.configs()
    print("grids", [c.grid[0] for c in cfgs], "P", [c.P for c in cfgs], "xi", [round(c.xi, 3) for c in cfgs])
    for rep in range(3):
        x = wl.force_moments(int(offs[-1]), 40 + rep)
        y = plan.apply(_t(x)).cpu().numpy()
        # eager work between replays
        z = torch.randn(1000, device="cuda:0") * 2.0
        torch.cuda.synchronize()
        del z
        for k, s in enumerate(sus):
            yi = _individual(lib, s, cfgs[k], x[offs[k]:offs[k + 1]])
            # the same kernels on the same data, except that a small
            # suspension's FP64 pair sum runs a thread per sphere inside the
            # batch and a wavefront per sphere alone: equal up to the order
            # of FP64 additions
            yb = y[offs[k]:offs[k + 1]]
            assert np.linalg.norm(yb - yi) <= 1e-13 * np.linalg.norm(yi), (rep, k)
    plan.close()
    eng.close()


def test_batch_autotuned_accuracy(lib, systems):
    sus, offs, pos, rad = systems
    eng = lib.Seasd(0, precision=lib.SEASD_FP32)
    plan = lib.Batch(eng, offs, _t(pos), _t(rad), [s.box for s in sus], target=1e-6)
    x = wl.force_moments(int(offs[-1]), 7)
    y = plan.apply(_t(x)).cpu().numpy()
    for k in (0, 3):
        s = sus[k]
        yo = ewald.apply(s.pos, s.radius, s.box, x[offs[k]:offs[k + 1]],
                         ewald.converged_params(s.box, s.radius, xi=0.5, tol_exp=6.5))
        err = np.linalg.norm(y[offs[k]:offs[k + 1]] - yo) / np.linalg.norm(yo)
        print(f"system {k}: N={s.n} L={s.L:.2f} rel err {err:.2e}")
        assert err < 2e-6
    plan.close()
    eng.close()


def test_batch_members_against_oracle(lib):
    """Three members of the benchmark's own many-suspension generator
    (workloads.batch_member; N = 1780, 7632 and 4540) that the autotuner puts
    on 64^3, 128^3 and 128^3 grids for a 1e-6 target, in one batched plan: each
    member's result at 64 sampled spheres against the FP64 oracle
    (tests/golden/batch_oracle_sample.npz, written by
    tests/golden/make_batch_sample.py from the oracle alone)."""
    import os
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.join(here, "golden"))
    import make_batch_sample as mk
    d = np.load(os.path.join(here, "golden", "batch_oracle_sample.npz"))
    sus, xs = [], []
    for k in mk.MEMBERS:
        s, x = mk.member_inputs(k)
        np.testing.assert_allclose([s.pos.sum(), (s.pos ** 2).sum()], d[f"pos_checksum_{k}"], rtol=1e-12)
        np.testing.assert_allclose([x.sum(), (x ** 2).sum()], d[f"x_checksum_{k}"], rtol=1e-12)
        sus.append(s)
        xs.append(x)
    offs = np.concatenate([[0], np.cumsum([s.n for s in sus])])
    eng = lib.Seasd(0, precision=lib.SEASD_FP32)
    plan = lib.Batch(eng, offs, _t(np.concatenate([s.pos for s in sus])),
                     _t(np.concatenate([s.radius for s in sus])), [s.box for s in sus], target=1e-6)
    grids = [c.grid[0] for c in plan.configs()]
    assert grids == [64, 128, 128]
    y = plan.apply(_t(np.concatenate(xs))).cpu().numpy()
    plan.close()
    eng.close()
    for j, k in enumerate(mk.MEMBERS):
        tg, yo = d[f"targets_{k}"], d[f"y_{k}"]
        yk = y[offs[j]:offs[j + 1]][tg]
        err = float(np.linalg.norm(yk - yo) / np.linalg.norm(yo))
        print(f"member {k}: N={sus[j].n} grid {grids[j]}^3 sample error {err:.3e}")
        assert np.all(np.isfinite(yk))
        assert err < 1e-6
