"""The paper's near-field / far-field hydrodynamic solve for a given
near-field resistance (Sec. 4.1, eqs. HI-nf, HI-ff, HI-solve, fM-comp).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Per sphere the unknowns are the far-field hydrodynamic force and torque
F (6 components), the far-field stresslet S (5, traceless, orthonormal basis)
and the velocity U (translational and rotational, 6). Given the near-field
force-velocity resistance R (6N x 6N, symmetric positive semi-definite), the
interparticle plus near-field strain forces Fp (6N) and the imposed strain
E (5N), they satisfy
  eq. HI-nf:  0 = -R U + F + Fp
  eq. HI-ff:  [U; -E] = -M [F; S]
with M the force-torque-stresslet (11N x 11N) block of the grand mobility
(oracle.ewald, whose inputs are the moments the spheres exert on the fluid,
so the paper's M maps -[F; S] to [U; -E] as written).

* direct_solve: the two equations as one dense linear system in (U, F, S).
* hi_solve: the paper's route. With R~ = R + lam I and the block operator
  D = diag(R~^-1, 0) on the 11N vectors, the unknown y = [F + lam U; S] solves
    (eq. fM-comp)  Mt y = rhs,   Mt = (I - lam M) D + M,
    (eq. HI-solve) rhs = (lam M - I) D [Fp; 0] + [0; E],
  then U = R~^-1 (y_F + Fp) and F = y_F - lam U.
The result does not depend on lam (a shift that keeps R~ invertible).

Vectors use the per-sphere interleaved order: 11 entries (F, T, S1..S5)
per sphere for the 11N vectors, 6 (F, T) for the 6N ones.
"""
from __future__ import annotations

import numpy as np

from . import ewald


def mobility_fts(pos, rad, box, params=None) -> np.ndarray:
    """The 11N x 11N force-torque-stresslet block of M (per-sphere order)."""
    n = pos.shape[0]
    M = ewald.dense_matrix(pos, rad, box, params).reshape(n, 12, n, 12)
    return M[:, :11, :, :11].reshape(11 * n, 11 * n)


def _ft_index(n):
    """Indices of the force-torque entries of an 11N vector."""
    return (np.arange(n)[:, None] * 11 + np.arange(6)[None, :]).reshape(-1)


def _s_index(n):
    return (np.arange(n)[:, None] * 11 + 6 + np.arange(5)[None, :]).reshape(-1)


def direct_solve(M11, R, Fp, E):
    """(U [n, 6], F [n, 6], S [n, 5]) from eqs. HI-nf and HI-ff as one system."""
    n = Fp.shape[0]
    ft, sx = _ft_index(n), _s_index(n)
    Mff, Mfs = M11[np.ix_(ft, ft)], M11[np.ix_(ft, sx)]
    Msf, Mss = M11[np.ix_(sx, ft)], M11[np.ix_(sx, sx)]
    n6, n5 = 6 * n, 5 * n
    A = np.zeros((2 * n6 + n5, 2 * n6 + n5))
    rhs = np.zeros(2 * n6 + n5)
    # -R U + F = -Fp
    A[:n6, :n6] = -R
    A[:n6, n6:2 * n6] = np.eye(n6)
    rhs[:n6] = -Fp.reshape(-1)
    # U + M_ff F + M_fs S = 0
    A[n6:2 * n6, :n6] = np.eye(n6)
    A[n6:2 * n6, n6:2 * n6] = Mff
    A[n6:2 * n6, 2 * n6:] = Mfs
    # M_sf F + M_ss S = E
    A[2 * n6:, n6:2 * n6] = Msf
    A[2 * n6:, 2 * n6:] = Mss
    rhs[2 * n6:] = E.reshape(-1)
    z = np.linalg.solve(A, rhs)
    return z[:n6].reshape(n, 6), z[n6:2 * n6].reshape(n, 6), z[2 * n6:].reshape(n, 5)


def hi_solve(M11, R, Fp, E, lam):
    """The same unknowns by eqs. HI-solve and fM-comp with the shift lam."""
    n = Fp.shape[0]
    ft, sx = _ft_index(n), _s_index(n)
    Rt_inv = np.linalg.inv(R + lam * np.eye(6 * n))
    D = np.zeros((11 * n, 11 * n))
    D[np.ix_(ft, ft)] = Rt_inv
    I = np.eye(11 * n)
    Mt = (I - lam * M11) @ D + M11
    p = np.zeros(11 * n)
    p[ft] = Fp.reshape(-1)
    e = np.zeros(11 * n)
    e[sx] = E.reshape(-1)
    rhs = (lam * M11 - I) @ (D @ p) + e
    y = np.linalg.solve(Mt, rhs)
    yF = y[ft]
    U = Rt_inv @ (yF + Fp.reshape(-1))
    F = yF - lam * U
    return U.reshape(n, 6), F.reshape(n, 6), y[sx].reshape(n, 5)


def pair_resistance(pos, rad, box, cut: float = 2.5, seed: int = 0) -> np.ndarray:
    """A synthetic near-field resistance with the structure of pairwise
    lubrication (the paper's resistance functions are not reproduced): every
    pair closer than cut (a_i + a_j)/2 adds squeeze and shear terms
    alpha n n^T + beta (I - n n^T) acting on U_i - U_j, and a rotational term
    gamma (I - n n^T) on Omega_i - Omega_j, with coefficients growing like
    1/(gap) near contact. The result is symmetric positive semi-definite by
    construction (a sum of Gram forms of velocity differences)."""
    n = pos.shape[0]
    inv = np.linalg.inv(box)
    R = np.zeros((6 * n, 6 * n))
    for i in range(n):
        for j in range(i + 1, n):
            d = pos[i] - pos[j]
            t = inv @ d
            d = box @ (t - np.round(t))
            r = float(np.linalg.norm(d))
            s = 2.0 * r / (rad[i] + rad[j])
            if s >= cut:
                continue
            nv = d / r
            nn = np.outer(nv, nv)
            gap = max(s - 2.0, 1e-3)
            a_ = 0.5 * (rad[i] + rad[j])
            blocks = [(0, (1.0 / gap) * 6.0 * np.pi * a_ * nn + 0.5 * np.log(1.0 / gap) * np.pi * a_ * (np.eye(3) - nn)),
                      (3, 0.4 * np.log(1.0 / gap) * np.pi * a_ ** 3 * (np.eye(3) - nn))]
            for off, B in blocks:
                ii, jj = 6 * i + off, 6 * j + off
                R[ii:ii + 3, ii:ii + 3] += B
                R[jj:jj + 3, jj:jj + 3] += B
                R[ii:ii + 3, jj:jj + 3] -= B
                R[jj:jj + 3, ii:ii + 3] -= B
    return R
