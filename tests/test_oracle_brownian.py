"""Pins of the Brownian far-field oracle (Sec. 4.3, eqs. br-f-ff, ivp-1,
ivp-forward, ivp-backward): A^(-1/2) c by eigendecomposition and by the
paper's initial value problem.

Checks fixed by the mathematics, not by the oracle's own formulas:
* applying A^(-1/2) twice and then A returns c;
* for A = alpha I both give c / sqrt(alpha), and A = I leaves c unchanged;
* the IVP march converges to the eigendecomposition result as dtau -> 0,
  at least at first order, and is already close at the paper's dtau = 0.1;
* for the scaled mobility, F = M^(-1/2) psi satisfies F^T M F = psi^T psi.
"""
import math

import numpy as np
import pytest

from oracle import brownian, ewald
from paper_1506_08481_amd import workloads as wl


def _spd(n, cond, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.exp(np.linspace(0.0, math.log(cond), n))
    return (Q * lam) @ Q.T


def test_inverse_sqrt_squares_to_the_inverse():
    A = _spd(30, 50.0, 1)
    c = np.random.default_rng(2).standard_normal(30)
    x = brownian.inverse_sqrt_apply(A, brownian.inverse_sqrt_apply(A, c))
    assert np.linalg.norm(A @ x - c) < 1e-12 * np.linalg.norm(c)
    assert c @ brownian.inverse_sqrt_apply(A, c) > 0


@pytest.mark.parametrize("alpha", [1.0, 0.2, 7.5])
def test_scalar_multiple_of_identity(alpha):
    c = np.random.default_rng(3).standard_normal(12)
    A = alpha * np.eye(12)
    assert np.allclose(brownian.inverse_sqrt_apply(A, c), c / math.sqrt(alpha), rtol=1e-14, atol=0)
    x = brownian.ivp_inverse_sqrt(A, c, 0.01)
    assert np.linalg.norm(x - c / math.sqrt(alpha)) < 2e-3 * np.linalg.norm(c) / math.sqrt(alpha)
    if alpha == 1.0:
        assert np.array_equal(brownian.ivp_inverse_sqrt(A, c, 0.1), c)


def test_ivp_converges_to_the_inverse_square_root():
    A = _spd(40, 20.0, 4)
    c = np.random.default_rng(5).standard_normal(40)
    exact = brownian.inverse_sqrt_apply(A, c)
    errs = [np.linalg.norm(brownian.ivp_inverse_sqrt(A, c, d) - exact) / np.linalg.norm(exact)
            for d in (0.2, 0.1, 0.05, 0.025)]
    assert all(e1 < e0 / 1.8 for e0, e1 in zip(errs, errs[1:]))
    assert errs[1] < 0.02


def test_mobility_brownian_force_reproduces_the_noise_norm():
    s = wl.bidisperse(6, 0.2, 71)
    psi = wl.force_moments(s.n, 72)
    p = ewald.converged_params(s.box, s.radius, xi=0.8)
    F = brownian.brownian_farfield(s.pos, s.radius, s.box, psi, None, params=p)
    M11 = brownian.incompressible_block(s.pos, s.radius, s.box, p)
    f = F[:, :11].reshape(-1)
    c = psi[:, :11].reshape(-1)
    assert abs(f @ M11 @ f - c @ c) < 1e-11 * (c @ c)
    assert np.all(F[:, 11] == 0.0)
    # the IVP at the paper's step agrees closely with the definition
    Fi = brownian.brownian_farfield(s.pos, s.radius, s.box, psi, 0.1, params=p)
    assert np.linalg.norm(Fi - F) / np.linalg.norm(F) < 0.02
