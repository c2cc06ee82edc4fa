"""Far-field Brownian forces through the inverse square root of the mobility.

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the library.

The far-field Brownian force moments are (2 kT / dt) times M^(-1/2) applied
to a unit Gaussian noise vector (Sec. 4.3, eq. br-f-ff). Two plain dense
versions of A^(-1/2) c, for a symmetric positive definite A:

* inverse_sqrt_apply: the definition, through the eigendecomposition
  A = Q diag(lambda) Q^T, A^(-1/2) c = Q diag(lambda^(-1/2)) Q^T c;
* ivp_inverse_sqrt: the paper's initial value problem (eq. ivp-1),
  dx/dtau = -(1/2) [tau I + (1 - tau) A]^(-1) (A - I) x, x(0) = c, whose
  solution at tau = 1 is A^(-1/2) c, marched in steps of dtau, each a forward
  Euler half step (eq. ivp-forward) followed by a backward Euler half step
  (eq. ivp-backward), every linear system solved densely.

brownian_farfield applies the IVP to the incompressible 11 x 11 block of the
grand mobility made dimensionless with the Stokes drag of the smallest
sphere, A = 6 pi eta a_min M, and scales back: M^(-1/2) c = sqrt(6 pi eta
a_min) A^(-1/2) c. (The paper writes the IVP for a mobility that is already
dimensionless; the scale is this build's reading, stated in its design notes.)
"""
from __future__ import annotations

import math

import numpy as np

from . import ewald


def inverse_sqrt_apply(A: np.ndarray, c: np.ndarray) -> np.ndarray:
    w, Q = np.linalg.eigh(0.5 * (A + A.T))
    if w.min() <= 0:
        raise ValueError("matrix is not positive definite")
    return Q @ ((Q.T @ c) / np.sqrt(w))


def ivp_inverse_sqrt(A: np.ndarray, c: np.ndarray, dtau: float) -> np.ndarray:
    """x(1) of eq. ivp-1 by the half-step scheme of eqs. ivp-forward and
    ivp-backward with K = round(1/dtau) steps of dtau = 1/K."""
    K = max(1, int(round(1.0 / dtau)))
    dt = 1.0 / K
    n = A.shape[0]
    I = np.eye(n)
    x = np.array(c, dtype=np.float64)
    for i in range(K):
        t0, t1 = i * dt, (i + 1) * dt
        # forward half step: (x' - x_i)/(dt/2) = -(1/2) [t0 I + (1 - t0) A]^-1 (A - I) x_i
        x_half = x - 0.25 * dt * np.linalg.solve(t0 * I + (1.0 - t0) * A, (A - I) @ x)
        # backward half step: (x_(i+1) - x')/(dt/2) = -(1/2) [t1 I + (1 - t1) A]^-1 (A - I) x_(i+1),
        # i.e. [K1 + (dt/4)(A - I)] x_(i+1) = K1 x'  with K1 = t1 I + (1 - t1) A
        K1 = t1 * I + (1.0 - t1) * A
        x = np.linalg.solve(K1 + 0.25 * dt * (A - I), K1 @ x_half)
    return x


def incompressible_block(pos, radius, box, params=None) -> np.ndarray:
    """The 11N x 11N force-torque-stresslet block of the grand mobility."""
    M = ewald.dense_matrix(pos, radius, box, params)
    n = pos.shape[0]
    return M.reshape(n, 12, n, 12)[:, :11, :, :11].reshape(11 * n, 11 * n)


def brownian_farfield(pos, radius, box, psi, dtau: float | None, eta: float = 1.0, params=None) -> np.ndarray:
    """M^(-1/2) psi on the 11 incompressible components ([n, 12] in, trace
    column 0 out). dtau None: the exact inverse square root; else the IVP."""
    n = pos.shape[0]
    M11 = incompressible_block(pos, radius, box, params)
    s = 6.0 * math.pi * eta * float(np.min(radius))
    c = psi[:, :11].reshape(-1)
    A = s * M11
    xs = inverse_sqrt_apply(A, c) if dtau is None else ivp_inverse_sqrt(A, c, dtau)
    out = np.zeros((n, 12))
    out[:, :11] = (math.sqrt(s) * xs).reshape(n, 11)
    return out
