"""The allocation-free product (seasd_mobility_apply_static, workspace in the
library's static device array) against the allocating entry point
seasd_mobility_apply: two calls in a row, the second with fewer spheres, so
the second call runs on an array that still holds the first call's contents;
and the host-side rejection of an input the array cannot hold."""
import math

import numpy as np
import pytest

from paper_1506_08481_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_08481_amd import seasd
    return seasd


CASES = {
    "fp64-real": dict(grid=32, P=16, m=0.9 * math.sqrt(math.pi * 16), xi=0.5, rc_factor=4.0),
    "fp32-hybrid": dict(grid=64, P=13, m=0.9 * math.sqrt(math.pi * 13), xi=0.6, rc_factor=3.5,
                        precision=1, size_approach=1),
}


@pytest.mark.parametrize("case", list(CASES))
def test_static_matches_allocating_entry_point(lib, case):
    cfg = CASES[case]
    eng = lib.Seasd(0, **cfg)
    tol = 1e-13 if cfg.get("precision", 0) == 0 else 1e-6
    for n, phi, seed in ((600, 0.2, 9100), (150, 0.15, 9101)):   # second call smaller
        s = wl.bidisperse(n, phi, seed)
        x = wl.force_moments(s.n, seed + 1)
        P_, R_, X_ = _t(s.pos), _t(s.radius), _t(x)
        y_ref = eng.apply(P_, R_, s.box, X_)
        y_st = torch.full_like(X_, float("nan"))
        eng.apply_static(P_, R_, s.box, X_, y_st)
        torch.cuda.synchronize()
        a, b = y_st.cpu().numpy(), y_ref.cpu().numpy()
        rel = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        print(f"{case} n={s.n}: static vs allocating rel {rel:.3e}, max abs {np.abs(a - b).max():.3e}")
        assert np.all(np.isfinite(a))
        assert rel <= tol
    eng.close()


def test_static_rejects_oversized_input(lib):
    eng = lib.Seasd(0, grid=64, P=16, xi=0.5, rc_factor=4.0)
    n = 2_000_000   # about 1.7 GB of per-sphere buffers: refused before any work is queued
    pos = torch.zeros((n, 3), dtype=torch.float64, device="cuda:0")
    rad = torch.ones(n, dtype=torch.float64, device="cuda:0")
    x = torch.zeros((n, 12), dtype=torch.float64, device="cuda:0")
    y = torch.zeros_like(x)
    with pytest.raises(lib.SeasdError) as ei:
        eng.apply_static(pos, rad, np.eye(3) * 400.0, x, y)
    assert ei.value.code == lib.SEASD_E_SCRATCH
    eng.close()
