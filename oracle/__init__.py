"""FP64 CPU oracle for the periodic grand-mobility product and far-field solve.

TEST INFRASTRUCTURE ONLY. Only tests/, the smoke check in __graft_entry__.py
and the cpu_baseline leg of bench.py may import or run anything in this
package. The library (paper_1506_08481_amd) never imports it, and it imports
nothing from the library: the two share no code.

Contents:
  symbols  - Fourier symbols of the 12x12 mobility blocks from the Faxen laws
             and multipole expansion (Sec. 2).
  ewald    - classical Ewald sum of those blocks (Hasimoto split, Sec. 2.2-2.3):
             converged mode and split-diagnostic modes.
  solve    - dense far-field solve and block-diagonal preconditioner blocks
             (Sec. 4.2) for small N.
  mpnn     - the project's learned preconditioner network on top of those
             blocks (not in the paper): forward, loss and backward in FP64,
             with optional bfloat16 rounding of matrix-product operands.
  brownian - M^(-1/2) by eigendecomposition and by the paper's initial value
             problem (Sec. 4.3).
  mixed    - the near-field / far-field solve of Sec. 4.1 for a given
             near-field resistance: directly and by eqs. HI-solve, fM-comp.
"""
from . import symbols, ewald, solve, mpnn, brownian, mixed  # noqa: F401
