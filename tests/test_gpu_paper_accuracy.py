"""The paper's accuracy study (Sec. 5.1) on the HIP path, through the C ABI.

Baseline system of Sec. 5.1: N = 50 bidisperse spheres, phi = 0.05, size
ratio lambda = 2, number fraction x2 = 0.3 of large spheres, force, torque and
stresslet of every sphere drawn at random and rescaled to unit norm, lattice
a1 = (L, 0, 0), a2 = (gamma L, L, 0), a3 = (0, 0, L). The error measure is the
relative infinity norm of eq. err-E, per block (U, W, E and the trace row).

* The printed point (Sec. 5.1.2, fig. M64_err): M = 64, P = 21,
  r_c = 6 (a_i + a_j), xi a1 = 0.46, m = 8 gives e_inf,r(E) < 1e-9 against
  the converged Ewald sum; the bound is read from tests/golden.
* The wave-space error law (Sec. 5.1.1, eq. error-scale): at xi a1 = 0.1 and
  M = 64 the wave sum is converged on the grid's k-set, so the difference
  between the Spectral Ewald wave part and the oracle's wave sum over the same
  k-set is the window's interpolation error alone; at m = sqrt(pi P) it
  falls like exp(-P pi/2); the fitted slope is read from tests/golden.
* Sheared cells (gamma = 0.5) give the same accuracy as orthogonal ones
  (Sec. 5.1.1).
* Odd and even P: the window is centred either way (eq. fgg-exp).
"""
import math

import numpy as np
import pytest

from oracle import ewald
from paper_1506_08481_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def sheared_box(L, gamma):
    return np.array([[L, gamma * L, 0.0], [0.0, L, 0.0], [0.0, 0.0, L]])


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_08481_amd import seasd
    return seasd


def baseline_system():
    """N = 50, phi = 0.05, lambda = 2, x2 = 0.3 (y2 = x2 lambda^3 / (x2 lambda^3 + 1 - x2))."""
    lam3 = 8.0
    y2 = 0.3 * lam3 / (0.3 * lam3 + 0.7)
    s = wl.bidisperse(50, 0.05, 5100, a1=1.0, a2=2.0, y2=y2)
    x = wl.unit_norm_moments(s.n, 5101)
    return s, x


BLOCKS = {"U": slice(0, 3), "W": slice(3, 6), "E": slice(6, 11), "e": slice(11, 12)}


def einf(y, yref):
    """eq. err-E per block: max over spheres of |y_i - y*_i| / |y*_i|."""
    out = {}
    for k, sl in BLOCKS.items():
        num = np.linalg.norm(y[:, sl] - yref[:, sl], axis=1)
        den = np.linalg.norm(yref[:, sl], axis=1)
        out[k] = float(np.max(num / den))
    return out


def gpu_apply(lib, s, box, x, **cfg):
    eng = lib.Seasd(0, **cfg)
    y = eng.apply(_t(s.pos), _t(s.radius), box, _t(x))
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    eng.close()
    return out


@pytest.fixture(scope="module")
def base():
    return baseline_system()


@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_printed_accuracy_point(lib, base, paper, gamma):
    s, x = base
    box = sheared_box(s.L, gamma)
    if gamma:
        s = wl.in_cell(s, box)
    yref = ewald.apply(s.pos, s.radius, box, x, ewald.converged_params(box, s.radius, xi=0.5, tol_exp=6.5))
    # the paper's runs of Sec. 5.1.2 use the hybrid size approach
    y = gpu_apply(lib, s, box, x, grid=64, P=21, m=8.0, xi=0.46, rc_factor=6.0, size_approach=lib.SEASD_SIZE_HYBRID)
    e = einf(y, yref)
    print(f"gamma={gamma} M=64 P=21 xi a1=0.46 m=8 rc=6(ai+aj) hybrid: einf {e}")
    bound = paper("printed_accuracy_einf_E")
    assert e["E"] < bound
    if gamma == 0.0:   # the printed case (orthogonal cell): the strain block is the most stringent
        assert max(e.values()) < bound
    else:              # the sheared cell: same strain accuracy, other blocks within a factor 2
        assert max(e.values()) < 2.0 * bound


def _wave_error(lib, s, box, x, P, m, size_approach=0):
    p = ewald.EwaldParams(xi=0.1, rc=1.0, grid=(64, 64, 64), parts=ewald.PARTS_WAVE)
    yo = ewald.apply(s.pos, s.radius, box, x, p)
    y = gpu_apply(lib, s, box, x, grid=64, P=P, m=m, xi=0.1, rc_factor=6.0, parts=lib.SEASD_PARTS_WAVE,
                  size_approach=size_approach)
    return einf(y, yo)["E"]


def test_hybrid_more_accurate_per_point(lib, base):
    """Sec. 5.1.1: with the second derivatives of the read-out taken in k
    space, the hybrid approach reaches a given wave-space accuracy with fewer
    window points than the real-space approach (the paper needs 13 against 15
    points for 1e-4). At the same P the hybrid error is therefore lower, by
    roughly the exp(-pi/2)-per-point law over that difference."""
    s, x = base
    for P in (9, 13):
        m = math.sqrt(math.pi * P)
        er = _wave_error(lib, s, s.box, x, P, m, lib.SEASD_SIZE_REAL)
        eh = _wave_error(lib, s, s.box, x, P, m, lib.SEASD_SIZE_HYBRID)
        print(f"P={P}: wave einf(E) real {er:.3e} hybrid {eh:.3e}")
        assert eh < er


def test_wave_error_law(lib, base, paper):
    s, x = base
    Ps = [5, 7, 9, 11, 13]
    errs = [_wave_error(lib, s, s.box, x, P, math.sqrt(math.pi * P)) for P in Ps]
    slope = np.polyfit(Ps, np.log(errs), 1)[0]
    rate = paper("error_law_rate")
    print(f"wave-only einf(E) at m = sqrt(pi P): {dict(zip(Ps, errs))}, slope {slope:.3f} (law -{rate:.3f})")
    assert np.all(np.diff(np.log(errs)) < 0)
    assert abs(-slope / rate - 1.0) < 0.25


def test_sheared_wave_error_as_orthogonal(lib, base):
    s, x = base
    for P in (9, 13):
        m = math.sqrt(math.pi * P)
        e0 = _wave_error(lib, s, s.box, x, P, m)
        e5 = _wave_error(lib, s, sheared_box(s.L, 0.5), x, P, m)
        print(f"P={P}: wave einf(E) gamma=0 {e0:.3e} gamma=0.5 {e5:.3e}")
        assert e5 < 4.0 * e0 and e0 < 4.0 * e5


def test_odd_and_even_P(lib, base, paper):
    """The window is centred on the sphere for odd and for even P (eq. fgg-exp
    read as exactly P points), so the error of an odd P sits on the same
    exp(-P pi/2)-type line as its even neighbours (eq. error-scale): the
    strain error falls at every step of P, the even P = 16 lies on the line
    through P = 15 and 17 (within a factor 1.4), and the decay per point is
    within the range the wave-only law test allows."""
    s, x = base
    yref = ewald.apply(s.pos, s.radius, s.box, x, ewald.converged_params(s.box, s.radius, xi=0.5, tol_exp=6.5))
    errs = {}
    for P in (15, 16, 17):
        y = gpu_apply(lib, s, s.box, x, grid=64, P=P, m=0.9 * math.sqrt(math.pi * P), xi=0.5, rc_factor=6.0)
        errs[P] = einf(y, yref)
        print(f"P={P}: einf {errs[P]}")
    lE = {P: math.log(e["E"]) for P, e in errs.items()}
    assert lE[15] > lE[16] > lE[17]
    assert abs(lE[16] - 0.5 * (lE[15] + lE[17])) < math.log(1.4)
    rate = paper("error_law_rate")
    per_point = 0.5 * (lE[15] - lE[17])
    assert 0.5 * rate < per_point < 1.25 * rate
    for e in errs.values():   # every block improves with P like the strain block
        assert max(e.values()) < 5.0 * e["E"]
