"""Reference far-field solve and block-diagonal preconditioner blocks.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* The far-field problem with no lubrication part: find x with M x = b for all
  12N unknowns (the far-field relation eq. HI-ff of Sec. 4.1 with the
  near-field resistance set to zero). Solved here by a dense LU solve of the
  oracle's matrix (small N).
* The block-diagonal approximation of M (Sec. 4.2): each sphere's 12x12 block
  with only its own periodic images, by direct Ewald summation; with no
  near-field part the incomplete LU of a block-diagonal matrix is its exact
  block LU, so the preconditioner is the per-sphere block inverse.
"""
from __future__ import annotations

import numpy as np

from . import ewald


def dense_solve(pos, rad, box, b, params=None) -> np.ndarray:
    """x with M x = b for all 12N unknowns (every coupling two-way)."""
    M = ewald.dense_matrix(pos, rad, box, params)
    return np.linalg.solve(M, b.reshape(-1)).reshape(b.shape)


def one_way_solve(pos, rad, box, b, params=None, compressible: bool = True) -> np.ndarray:
    """The far-field solve with the paper's one-way pressure-moment coupling
    (Sec. 2.3: the interaction part of a pressure moment is evaluated only after
    F, T and S are known; Sec. 4.1 solves for F and S only):
      s_self = b_trace / m_self             (own trace equation, no interactions)
      A f    = b_f - C s_self               (A: 11x11 incompressible block,
                                             C: velocity/strain of the sources)
      s      = (b_trace - D f) / m_self     (pressure Faxen law; D: pressure row)
    With compressible=False the trace is dropped: A f = b_f and s = 0."""
    N = pos.shape[0]
    M = ewald.dense_matrix(pos, rad, box, params).reshape(N, 12, N, 12)
    A = M[:, :11, :, :11].reshape(11 * N, 11 * N)
    bf = b[:, :11].reshape(-1)
    x = np.zeros_like(b)
    if compressible:
        m_self = np.array([M[i, 11, i, 11] for i in range(N)])
        s_self = b[:, 11] / m_self
        C = M[:, :11, :, 11].reshape(11 * N, N)
        f = np.linalg.solve(A, bf - C @ s_self)
        D = M[:, 11, :, :11].reshape(N, 11 * N)
        x[:, :11] = f.reshape(N, 11)
        x[:, 11] = (b[:, 11] - D @ f) / m_self
    else:
        x[:, :11] = np.linalg.solve(A, bf).reshape(N, 11)
    return x


def self_image_block(a: float, box, params=None) -> np.ndarray:
    """M_ii for one sphere of radius a alone in the periodic box."""
    pos = np.zeros((1, 3))
    rad = np.array([a])
    return ewald.dense_matrix(pos, rad, np.asarray(box, dtype=np.float64), params)
