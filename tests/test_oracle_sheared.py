"""Pins of the FP64 oracle in sheared cells (lattice a1 = (L, 0, 0),
a2 = (gamma L, L, 0), a3 = (0, 0, L); Sec. 3.2, eq. non-ortho-shape, and the
sheared accuracy runs of Sec. 5.1).

The oracle sums over a general lattice (image shifts from the cell heights,
k = B q with B = 2 pi A^-T). Nothing here compares it with itself:
* gamma = 1 and gamma = -1 generate the same lattice as the cube, so the
  periodic sum must equal the cubic one although every image and wave vector
  is enumerated differently;
* the split parameter xi must drop out;
* a mirror x -> -x maps the cell of strain gamma onto the cell of strain
  -gamma, and the product must map with it (vectors, pseudovectors and
  tensors transformed);
* the incompressible 11 x 11 block stays symmetric and positive definite.
"""
import numpy as np
import pytest

from oracle import ewald, symbols
from paper_1506_08481_amd import workloads as wl


def sheared_box(L, gamma):
    return np.array([[L, gamma * L, 0.0], [0.0, L, 0.0], [0.0, 0.0, L]])


@pytest.fixture(scope="module")
def susp():
    s = wl.bidisperse(8, 0.15, 51)
    return s, wl.force_moments(s.n, 52)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("gamma", [1.0, -1.0])
def test_unit_strain_is_the_cubic_lattice(susp, gamma):
    s, x = susp
    p = ewald.converged_params(s.box, s.radius, xi=0.6)
    y0 = ewald.apply(s.pos, s.radius, s.box, x, p)
    y1 = ewald.apply(s.pos, s.radius, sheared_box(s.L, gamma), x, p)
    assert _rel(y1, y0) < 1e-12


def test_xi_independence_sheared(susp):
    s, x = susp
    box = sheared_box(s.L, 0.5)
    ys = [ewald.apply(s.pos, s.radius, box, x, ewald.converged_params(box, s.radius, xi=xi))
          for xi in (0.45, 0.8)]
    assert _rel(ys[1], ys[0]) < 1e-13
    # and the strain matters: the sheared lattice is not the cubic one
    yc = ewald.apply(s.pos, s.radius, s.box, x, ewald.converged_params(s.box, s.radius, xi=0.6))
    assert _rel(ys[0], yc) > 1e-4


def _mirror_moments(x):
    """x -> -x mirror: vectors flip their x component, pseudovectors (torque,
    spin) the other two, symmetric tensors transform as R S R^T."""
    R = np.diag([-1.0, 1.0, 1.0])
    out = x.copy()
    out[:, 0:3] = x[:, 0:3] @ R.T
    out[:, 3:6] = -(x[:, 3:6] @ R.T)
    Y = symbols.traceless_basis()
    S = np.einsum("nm,mab->nab", x[:, 6:11], Y)
    S = np.einsum("ac,ncd,bd->nab", R, S, R)
    out[:, 6:11] = np.einsum("mab,nab->nm", Y, S)
    return out


def test_mirror_maps_strain_to_minus_strain(susp):
    s, x = susp
    gamma = 0.5
    box = sheared_box(s.L, gamma)
    p = ewald.converged_params(box, s.radius, xi=0.6)
    y = ewald.apply(s.pos, s.radius, box, x, p)
    R = np.diag([-1.0, 1.0, 1.0])
    ym = ewald.apply(s.pos @ R.T, s.radius, sheared_box(s.L, -gamma), _mirror_moments(x), p)
    assert _rel(ym, _mirror_moments(y)) < 1e-13


def test_symmetric_positive_definite_sheared():
    s = wl.bidisperse(6, 0.2, 61)
    box = sheared_box(s.L, 0.5)
    M = ewald.dense_matrix(s.pos, s.radius, box, ewald.converged_params(box, s.radius, xi=0.8))
    n = s.n
    A = M.reshape(n, 12, n, 12)[:, :11, :, :11].reshape(11 * n, 11 * n)
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
