"""Pins of the near-field / far-field solve oracle (oracle/mixed.py; Sec. 4.1,
eqs. HI-nf, HI-ff, HI-solve, fM-comp).

Checks fixed by the physics and the algebra rather than by the oracle's own
formulas:
* one sphere per periodic cell (simple cubic array) with an isotropic
  near-field resistance r I: the drags add, U = Fp mu / (1 + r mu) with
  Hasimoto's array mobility mu for translation and the exact rotating-array
  mobility for rotation;
* one sphere in a large cell in a pure strain with no near-field part: the
  stresslet is the single-sphere (20/3) pi eta a^3 E up to the (a/L)^3 image
  correction;
* with no near-field resistance the far-field forces balance the applied
  ones (F = -Fp);
* the paper's shifted formulation gives the direct solution of the two
  equations for any shift lam (the result does not depend on lam).
"""
import math

import numpy as np
import pytest

from oracle import ewald, mixed
from paper_1506_08481_amd import workloads as wl

HASIMOTO_SC = 2.837297


def _sc(a, L, xi=0.5):
    pos = np.zeros((1, 3))
    rad = np.array([a])
    box = np.eye(3) * L
    return pos, rad, box, mixed.mobility_fts(pos, rad, box, ewald.converged_params(box, rad, xi=xi, tol_exp=6.5))


@pytest.mark.parametrize("r", [0.0, 3.0, 40.0])
def test_sc_array_drags_add(r):
    a, L = 1.0, 9.0
    pos, rad, box, M11 = _sc(a, L)
    Fp = np.array([[0.7, -0.2, 0.4, 0.3, 0.1, -0.5]])
    R = r * np.eye(6)
    U, F, S = mixed.hi_solve(M11, R, Fp, np.zeros((1, 5)), lam=6.0 * math.pi * a)
    mu_t = (1.0 - HASIMOTO_SC * a / L + 4.0 * math.pi / 3.0 * (a / L) ** 3) / (6.0 * math.pi * a)
    mu_r = (1.0 - 4.0 * math.pi / 3.0 * (a / L) ** 3) / (8.0 * math.pi * a ** 3)
    np.testing.assert_allclose(U[0, :3], Fp[0, :3] * mu_t / (1.0 + r * mu_t), rtol=2e-7)
    np.testing.assert_allclose(U[0, 3:], Fp[0, 3:] * mu_r / (1.0 + r * mu_r), rtol=1e-11)
    np.testing.assert_allclose(F[0], R @ U[0] - Fp[0], atol=1e-12)   # eq. HI-nf
    assert np.max(np.abs(S)) < 1e-12                                  # cubic symmetry


def test_single_sphere_in_strain():
    """The stresslet tends to the single-sphere value as the cell grows, the
    image correction falling like (a/L)^3 (the strain of a stresslet lattice
    at the sphere scales with the number density)."""
    a = 1.0
    E = np.array([[0.3, -0.8, 0.2, 0.5, -0.1]])
    S0 = 20.0 / 3.0 * math.pi * a ** 3 * E
    rel = {}
    for L in (40.0, 80.0):
        # the converged sum does not depend on xi; xi L fixed keeps the
        # number of wave vectors the same for both cells
        pos, rad, box, M11 = _sc(a, L, xi=10.0 / L)
        U, F, S = mixed.hi_solve(M11, np.zeros((6, 6)), np.zeros((1, 6)), E, lam=6.0 * math.pi * a)
        assert np.max(np.abs(F)) < 1e-12 and np.max(np.abs(U)) < 1e-12
        rel[L] = np.linalg.norm(S - S0) / np.linalg.norm(S0)
    assert rel[80.0] < 1e-4
    assert abs(rel[40.0] / rel[80.0] / 8.0 - 1.0) < 0.05


@pytest.fixture(scope="module")
def cluster():
    s = wl.bidisperse(8, 0.25, 8100)
    p = ewald.converged_params(s.box, s.radius, xi=0.6, tol_exp=6.5)
    M11 = mixed.mobility_fts(s.pos, s.radius, s.box, p)
    R = mixed.pair_resistance(s.pos, s.radius, s.box, cut=3.0)
    rng = np.random.default_rng(8101)
    Fp = rng.standard_normal((s.n, 6))
    E = rng.standard_normal((s.n, 5))
    return s, M11, R, Fp, E


def test_synthetic_resistance_is_psd_with_pairs(cluster):
    s, M11, R, Fp, E = cluster
    assert np.abs(R).max() > 0.0                      # some pairs are within the cut
    assert np.allclose(R, R.T)
    assert np.linalg.eigvalsh(R).min() > -1e-10 * np.abs(R).max()


@pytest.mark.parametrize("lam_scale", [1.0, 0.1, 25.0])
def test_shifted_formulation_equals_direct_solve(cluster, lam_scale):
    s, M11, R, Fp, E = cluster
    U0, F0, S0 = mixed.direct_solve(M11, R, Fp, E)
    lam = lam_scale * 6.0 * math.pi * float(s.radius.min())
    U, F, S = mixed.hi_solve(M11, R, Fp, E, lam)
    for a, b in ((U, U0), (F, F0), (S, S0)):
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)
    # the solution satisfies both equations of the paper
    assert np.linalg.norm(-R @ U.reshape(-1) + F.reshape(-1) + Fp.reshape(-1)) < 1e-10 * np.linalg.norm(Fp)
    y = np.concatenate([F, S], axis=1).reshape(-1)
    lhs = np.concatenate([U, -E], axis=1).reshape(-1)
    assert np.linalg.norm(lhs + M11 @ y) < 1e-10 * np.linalg.norm(lhs)


def test_no_resistance_forces_balance(cluster):
    s, M11, R, Fp, E = cluster
    U, F, S = mixed.hi_solve(M11, np.zeros_like(R), Fp, E, lam=6.0 * math.pi)
    np.testing.assert_allclose(F, -Fp, atol=1e-11 * np.abs(Fp).max())
