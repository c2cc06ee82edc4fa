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
    M = ewald.dense_matrix(pos, rad, box, params)
    return np.linalg.solve(M, b.reshape(-1)).reshape(b.shape)


def self_image_block(a: float, box, params=None) -> np.ndarray:
    """M_ii for one sphere of radius a alone in the periodic box."""
    pos = np.zeros((1, 3))
    rad = np.array([a])
    return ewald.dense_matrix(pos, rad, np.asarray(box, dtype=np.float64), params)
