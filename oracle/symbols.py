"""Fourier symbols of the 12x12 grand-mobility blocks, built by polynomial algebra.

TEST INFRASTRUCTURE ONLY: the oracle is imported by tests/, the smoke check and
the CPU-baseline leg of the benchmark, never by the library.

What is built here (Sec. 2.1-2.3 of the paper):

* The force density a sphere j puts into the fluid, as a Fourier amplitude per
  wave vector k (the phase exp(i k.r_j) left out), for each of its 11
  incompressible force moments. The force carries the Faxen factor
  (1 - a_j^2 k^2/6) of the multipole expansion (eq. mul-expand); the torque is
  the curl of a point torque density, -(i/2) k x T; the traceless stresslet is
  the divergence of a point stresslet density with the (1 - a_j^2 k^2/10)
  factor of eq. faxen-s.
* The read-out at sphere i, by the Faxen laws (eqs. faxen-f, faxen-t, faxen-s):
  (1 - a_i^2 k^2/6) on the velocity, half the curl for the spin, and
  (1 - a_i^2 k^2/10) times the symmetric gradient for the rate of strain.
* The incompressible Stokes propagator (I k^2 - k k)/(eta k^4), the Fourier form
  of the periodic Oseen tensor (eq. oseen-peridoic).
* The compressible-solvent couplings (Sec. 2.3): the pressure moment is a fluid
  source with velocity Q = r/(16 pi eta r^3), i.e. (i k)/(4 eta k^2) in Fourier
  form (eqs. pres-vel-disturb, wave-dist-S); the trace output row is the
  pressure Faxen law (eq. faxen-p) with the pressure of the force density,
  p = i k.f / k^2 (eqs. pres-funda, pres-distro).

Conventions (the paper's signs are not consistent with each other, so the
operator is fixed by physics and checked by symmetry, free-space closed forms
and xi-independence):
* inputs x = (F, T, S1..S5, s6) are the moments each sphere exerts on the
  fluid; S1..S5 are coordinates of the traceless stresslet in the orthonormal
  basis Y below and s6 = trace(S)/sqrt(3);
* outputs y = (U, Omega, E1..E5, e6): sphere velocity, spin, minus the
  ambient strain rate the sphere would need (the paper's -E row) in the same
  basis, and the matching trace coordinate of -E (e6 = -E_expansion/sqrt(3)).
  With these choices S:E is a plain dot product and the 11x11 incompressible
  block is symmetric positive definite.

Each block symbol is a polynomial in (k1, k2, k3, Ai, Aj) with Ai = a_i^2,
Aj = a_j^2, times one of two scalar Fourier kernels:
  "stokes":  1/k^4   (real-space partner -r/(8 pi))
  "laplace": 1/k^2   (real-space partner 1/(4 pi r))
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

NVAR = 5  # k1, k2, k3, Ai, Aj


class Poly:
    """Sparse polynomial with complex coefficients in (k1, k2, k3, Ai, Aj)."""

    __slots__ = ("t",)

    def __init__(self, t=None):
        self.t = {}
        if t:
            for m, c in t.items():
                if c != 0:
                    self.t[m] = complex(c)

    @staticmethod
    def const(c):
        return Poly({(0,) * NVAR: c})

    @staticmethod
    def var(i):
        e = [0] * NVAR
        e[i] = 1
        return Poly({tuple(e): 1.0})

    def __add__(self, o):
        o = o if isinstance(o, Poly) else Poly.const(o)
        r = dict(self.t)
        for m, c in o.t.items():
            r[m] = r.get(m, 0) + c
        return Poly({m: c for m, c in r.items() if c != 0})

    __radd__ = __add__

    def __neg__(self):
        return Poly({m: -c for m, c in self.t.items()})

    def __sub__(self, o):
        return self + (-(o if isinstance(o, Poly) else Poly.const(o)))

    def __rsub__(self, o):
        return Poly.const(o) - self

    def __mul__(self, o):
        if not isinstance(o, Poly):
            return Poly({m: c * o for m, c in self.t.items()})
        r = {}
        for m1, c1 in self.t.items():
            for m2, c2 in o.t.items():
                m = tuple(a + b for a, b in zip(m1, m2))
                r[m] = r.get(m, 0) + c1 * c2
        return Poly({m: c for m, c in r.items() if c != 0})

    __rmul__ = __mul__


def traceless_basis() -> np.ndarray:
    """Orthonormal (Frobenius) basis Y[0..4] of symmetric traceless 3x3 tensors."""
    s2, s6 = math.sqrt(2.0), math.sqrt(6.0)
    Y = np.zeros((5, 3, 3))
    Y[0] = np.diag([1.0, -1.0, 0.0]) / s2
    Y[1] = np.diag([-1.0, -1.0, 2.0]) / s6
    Y[2][0, 1] = Y[2][1, 0] = 1.0 / s2
    Y[3][0, 2] = Y[3][2, 0] = 1.0 / s2
    Y[4][1, 2] = Y[4][2, 1] = 1.0 / s2
    return Y


def levi_civita(a, b, c) -> int:
    return int(np.sign((b - a) * (c - a) * (c - b))) if len({a, b, c}) == 3 else 0


def _build(eta: float):
    K = [Poly.var(0), Poly.var(1), Poly.var(2)]
    Ai, Aj = Poly.var(3), Poly.var(4)
    k2 = K[0] * K[0] + K[1] * K[1] + K[2] * K[2]
    Y = traceless_basis()
    I = 1j
    zero = Poly()

    # force density amplitude for a unit input b (b < 11)
    spread = []
    for b in range(3):                                  # force
        spread.append([(1 - Aj * k2 * (1.0 / 6.0)) if al == b else zero for al in range(3)])
    for b in range(3):                                  # torque: -(i/2) k x e_b
        spread.append([sum((K[be] * (-0.5 * I * levi_civita(al, be, b)) for be in range(3)), zero)
                       for al in range(3)])
    for m in range(5):                                  # stresslet: i (1 - Aj k^2/10) Y_m k
        fac = (1 - Aj * k2 * 0.1) * I
        spread.append([fac * sum((K[be] * Y[m][al, be] for be in range(3)), zero) for al in range(3)])

    # read-out covectors acting on the velocity amplitude (a < 11)
    gather = []
    for a in range(3):                                  # velocity with Faxen factor
        gather.append([(1 - Ai * k2 * (1.0 / 6.0)) if al == a else zero for al in range(3)])
    for lam in range(3):                                # spin: (-i/2) (k x v)_lam
        gather.append([sum((K[be] * (-0.5 * I * levi_civita(lam, be, al)) for be in range(3)), zero)
                       for al in range(3)])
    for m in range(5):                                  # strain: -i (1 - Ai k^2/10) (Y_m k) . v
        fac = (1 - Ai * k2 * 0.1) * (-I)
        gather.append([fac * sum((K[be] * Y[m][al, be] for be in range(3)), zero) for al in range(3)])

    stokes = [[zero] * 12 for _ in range(12)]
    laplace = [[zero] * 12 for _ in range(12)]
    for a in range(11):
        for b in range(11):
            acc = zero
            for al in range(3):
                if not gather[a][al].t:
                    continue
                for be in range(3):
                    if not spread[b][be].t:
                        continue
                    prop = (k2 if al == be else zero) - K[al] * K[be]
                    acc = acc + gather[a][al] * prop * spread[b][be]
            stokes[a][b] = acc * (1.0 / eta)
    src = math.sqrt(3.0) / (4.0 * eta)
    for a in range(11):                                 # velocity of a fluid source, (i k)/(4 eta k^2)
        laplace[a][11] = sum((gather[a][al] * K[al] * (src * I) for al in range(3)), zero)
    for b in range(11):                                 # pressure Faxen row: -(sqrt3/4eta) i k.f/k^2
        laplace[11][b] = sum((K[al] * spread[b][al] * (-src * I) for al in range(3)), zero)
    return stokes, laplace


@lru_cache(maxsize=4)
def block_symbols(eta: float = 1.0):
    """Return, per kernel family, (alphas, C) where alphas is an [n, 3] int array
    of k-exponents and C is [n, 2, 2, 12, 12] complex: the coefficient of
    k^alpha * Ai^p * Aj^q in block (a, b)."""
    stokes, laplace = _build(eta)
    out = {}
    for name, blocks in (("stokes", stokes), ("laplace", laplace)):
        keys = sorted({m[:3] for a in range(12) for b in range(12) for m in blocks[a][b].t})
        idx = {k: n for n, k in enumerate(keys)}
        C = np.zeros((len(keys), 2, 2, 12, 12), dtype=np.complex128)
        for a in range(12):
            for b in range(12):
                for m, c in blocks[a][b].t.items():
                    C[idx[m[:3]], m[3], m[4], a, b] += c
        out[name] = (np.array(keys, dtype=np.int64).reshape(-1, 3), C)
    return out


def self_mobility(a: float, eta: float = 1.0) -> np.ndarray:
    """Single-sphere mobility in the 12-component layout: the self terms of the
    Faxen laws (eqs. faxen-f, faxen-t, faxen-s) and of the pressure Faxen law
    (eq. faxen-p with S = -(16/3) pi eta a^3 E for an isolated sphere)."""
    d = np.empty(12)
    d[0:3] = 1.0 / (6.0 * math.pi * eta * a)
    d[3:6] = 1.0 / (8.0 * math.pi * eta * a ** 3)
    d[6:11] = 1.0 / (20.0 / 3.0 * math.pi * eta * a ** 3)
    d[11] = 1.0 / (16.0 / 3.0 * math.pi * eta * a ** 3)
    return np.diag(d)
