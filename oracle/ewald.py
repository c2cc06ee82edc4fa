"""Plain FP64 classical Ewald sum of the periodic grand mobility product y = M x.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of the benchmark; the library never calls it.

This is the paper's own yardstick: the Spectral Ewald result is measured
against a converged direct Ewald sum (Sec. 5.1, eq. err-E). It is not the Spectral Ewald method: there is no grid, no window
and no FFT. Every block symbol comes from oracle.symbols; this file only sums
them.

Split (Hasimoto, eqs. ewald-theta, oseen-ewald-rs, oseen-ewald-ws, source-split):
  y_i = sum over pairs and lattice images (not i=j at p=0) of the real-space
        blocks
      + (1/V) sum_{k != 0} exp(-i k.r_i) sum_j K(k) exp(i k.r_j) x_j
      - (continuum integral of the i=j wave-space symbol) x_i
      + single-sphere self mobility x_i.
Wave-space kernels: (1 + k^2/4xi^2) exp(-k^2/4xi^2)/k^4 (Stokes) and
exp(-k^2/4xi^2)/k^2 (Laplace). Their real-space complements are
  B_R(r)   = -(1/8pi) [ r erfc(xi r) - exp(-xi^2 r^2)/(xi sqrt(pi)) ]
  phi_R(r) = erfc(xi r)/(4 pi r),
and a symbol monomial k^alpha becomes the derivative (i d)^alpha of them.
Derivatives of a radial function f(r) are taken from its hierarchy
f_n = ((1/r) d/dr)^n f, with
  d^a/dx^a d^b/dy^b d^c/dz^c f = sum_{i,j,l} c(a,i) c(b,j) c(c,l)
        x^(a-2i) y^(b-2j) z^(c-2l) f_(a+b+c-i-j-l),
  c(n, i) = n! / (2^i i! (n-2i)!),
and for erfc(xi r)/r the hierarchy is the standard upward recurrence
  B_0 = erfc(xi r)/r,  B_n = [(2n-1) B_(n-1) + (2 xi^2)^n exp(-xi^2 r^2)/(xi sqrt(pi))]/r^2,
  ((1/r) d/dr)^n erfc(xi r)/r = (-1)^n B_n.

Pins (tests/test_oracle.py) fix every block of the sum against closed forms,
printed values, finite differences and invariances, the periodic images of
the velocity, spin, strain and pressure read-out rows included: the image
parts, for which the paper prints no value, are fixed by the identities the
exact periodic fields satisfy (Hasimoto's array, symmetry, the gradient and
curl relations between the read-outs, the source-flow divergence and Stokes'
equations between pressure and velocity).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree
from scipy.special import erfc, gamma

from .symbols import block_symbols, self_mobility

PARTS_REAL, PARTS_WAVE, PARTS_SELF = 1, 2, 4
PARTS_ALL = 7


@dataclass
class EwaldParams:
    xi: float                 # splitting parameter (Beenakker convention, Sec. 2.2)
    rc: float                 # real-space cutoff on |r_ij + R_p| (absolute length)
    kc: float | None = None   # wave-space cutoff on |k| (None: use the grid k-set)
    grid: tuple | None = None # (M1, M2, M3): wave sum over |q_d| < M_d/2 (Nyquist excluded)
    eta: float = 1.0
    parts: int = PARTS_ALL


def converged_params(box: np.ndarray, radius: np.ndarray, eta: float = 1.0,
                     xi: float | None = None, tol_exp: float = 8.0) -> EwaldParams:
    """Cutoffs for a converged sum: xi*rc = tol_exp and kc/(2 xi) = tol_exp, so
    both Gaussian tails are below exp(-tol_exp^2) (about 1.6e-28 for 8) before
    polynomial prefactors. The result does not depend on xi (tested)."""
    L = float(np.cbrt(abs(np.linalg.det(box))))
    if xi is None:
        xi = 4.0 / L if L > 12.0 else 0.5
    rc = tol_exp / xi
    kc = 2.0 * xi * tol_exp
    return EwaldParams(xi=xi, rc=rc, kc=kc, eta=eta)


# ---------------------------------------------------------------------------
# radial functions

def smith_B(r: np.ndarray, xi: float, nmax: int) -> np.ndarray:
    """B_0..B_nmax of erfc(xi r)/r; for xi = 0 these are (2n-1)!!/r^(2n+1)."""
    r = np.asarray(r, dtype=np.float64)
    out = np.empty((nmax + 1,) + r.shape)
    r2 = r * r
    if xi == 0.0:
        out[0] = 1.0 / r
        for n in range(1, nmax + 1):
            out[n] = (2 * n - 1) * out[n - 1] / r2
        return out
    out[0] = erfc(xi * r) / r
    g = np.exp(-xi * xi * r2) / (xi * math.sqrt(math.pi))
    for n in range(1, nmax + 1):
        out[n] = ((2 * n - 1) * out[n - 1] + (2.0 * xi * xi) ** n * g) / r2
    return out


def hierarchy(family: str, r: np.ndarray, xi: float, nmax: int) -> np.ndarray:
    """f_n = ((1/r) d/dr)^n f for n = 0..nmax (entry 0 is left as NaN: unused)."""
    B = smith_B(r, xi, nmax)
    f = np.full_like(B, np.nan)
    if family == "stokes":
        # f = -(1/8pi) chi, chi_1 = B_0, chi_n = (-1)^(n-1) B_(n-1)
        for n in range(1, nmax + 1):
            f[n] = -(1.0 / (8.0 * math.pi)) * ((-1.0) ** (n - 1)) * B[n - 1]
    else:
        for n in range(1, nmax + 1):
            f[n] = (1.0 / (4.0 * math.pi)) * ((-1.0) ** n) * B[n]
    return f


def _cn(n: int, i: int) -> float:
    return math.factorial(n) / (2 ** i * math.factorial(i) * math.factorial(n - 2 * i))


def radial_derivatives(d: np.ndarray, fh: np.ndarray, alphas: np.ndarray) -> np.ndarray:
    """d: [P, 3] displacements; fh: [nmax+1, P] hierarchy; alphas: [A, 3].
    Returns [P, A] with the partial derivative d^alpha f at each displacement."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    out = np.zeros((d.shape[0], alphas.shape[0]))
    for n, (a, b, c) in enumerate(alphas):
        acc = np.zeros(d.shape[0])
        for i in range(a // 2 + 1):
            for j in range(b // 2 + 1):
                for l in range(c // 2 + 1):
                    coef = _cn(a, i) * _cn(b, j) * _cn(c, l)
                    order = a + b + c - i - j - l
                    acc = acc + coef * x ** (a - 2 * i) * y ** (b - 2 * j) * z ** (c - 2 * l) * fh[order]
        out[:, n] = acc
    return out


# ---------------------------------------------------------------------------
# lattice helpers

def reciprocal(box: np.ndarray) -> np.ndarray:
    """B with B^T = 2 pi A^-1 (Sec. 2.2): columns are the reciprocal vectors."""
    return 2.0 * math.pi * np.linalg.inv(box).T


def k_vectors(box: np.ndarray, params: EwaldParams) -> np.ndarray:
    B = reciprocal(box)
    if params.grid is not None:
        M = params.grid
        rng = [np.arange(-(m // 2) + 1, (m + 1) // 2) if m % 2 == 0 else np.arange(-(m // 2), m // 2 + 1)
               for m in M]
        # |q_d| < M_d/2: the Nyquist plane of an even grid is excluded
        rng = [r[np.abs(r) < m / 2.0] for r, m in zip(rng, M)]
        q = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3)
    else:
        kc = params.kc
        nmax = [int(math.ceil(kc * np.linalg.norm(box[:, d]) / (2 * math.pi))) + 1 for d in range(3)]
        rng = [np.arange(-n, n + 1) for n in nmax]
        q = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3)
    q = q[np.any(q != 0, axis=1)]
    k = q @ B.T
    if params.grid is None:
        k = k[np.einsum("ij,ij->i", k, k) <= params.kc ** 2]
    return k


def image_shifts(box: np.ndarray, rc: float) -> np.ndarray:
    """Lattice vectors R_p that can bring a minimum-image displacement within rc."""
    V = abs(np.linalg.det(box))
    n = []
    for d in range(3):
        e, f = box[:, (d + 1) % 3], box[:, (d + 2) % 3]
        height = V / np.linalg.norm(np.cross(e, f))
        n.append(int(math.ceil(rc / height)) + 1)
    rng = [np.arange(-m, m + 1) for m in n]
    p = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3)
    return p @ box.T


# ---------------------------------------------------------------------------
# the three parts

def _wave_kernel(family: str, k2: np.ndarray, xi: float) -> np.ndarray:
    e = np.exp(-k2 / (4.0 * xi * xi))
    if family == "stokes":
        return (1.0 + k2 / (4.0 * xi * xi)) * e / (k2 * k2)
    return e / k2


def _source_premultiplied(C: np.ndarray, rad_j: np.ndarray, x: np.ndarray) -> np.ndarray:
    """X[j, alpha, p, a, col] = sum_{q,b} C[alpha, p, q, a, b] Aj^q x[j, b, col]."""
    Aj = rad_j ** 2
    xq = np.stack([x, Aj[:, None, None] * x], axis=1)          # [N, q, b, col]
    return np.einsum("npqab,jqbc->jnpac", C, xq, optimize=True)


def real_part(pos, rad, box, x, params: EwaldParams, targets=None) -> np.ndarray:
    """Real-space pair sum over all images with |r_i - r_j + R_p| < rc,
    excluding i = j at R_p = 0. x: [N, 12, C]."""
    N = pos.shape[0]
    tgt = np.arange(N) if targets is None else np.asarray(targets)
    syms = block_symbols(params.eta)
    out = np.zeros((tgt.shape[0], 12, x.shape[2]))
    shifts = image_shifts(box, params.rc)
    inv = np.linalg.inv(box)
    prepared = {}
    for fam in ("stokes", "laplace"):
        alphas, C = syms[fam]
        Cr = C * (1j) ** alphas.sum(1)[:, None, None, None, None]   # (i d)^alpha
        assert np.max(np.abs(Cr.imag)) < 1e-12
        prepared[fam] = (alphas, _source_premultiplied(Cr.real, rad, x), int(alphas.sum(1).max()))
    def accumulate(t0, ii, jj, dv):
        rv = np.linalg.norm(dv, axis=-1)
        Ai = rad[tgt[t0 + ii]] ** 2
        for fam in ("stokes", "laplace"):
            alphas, X, nmax = prepared[fam]
            fh = hierarchy(fam, rv, params.xi, nmax)
            D = radial_derivatives(dv, fh, alphas)                  # [P, A]
            Xs = X[jj]                                              # [P, A, p, a, col]
            contrib = np.einsum("pn,pnac->pac", D, Xs[:, :, 0]) + \
                Ai[:, None, None] * np.einsum("pn,pnac->pac", D, Xs[:, :, 1])
            np.add.at(out, t0 + ii, contrib)

    Ls = np.diag(box)
    orthorhombic = np.allclose(box, np.diag(Ls))
    if orthorhombic and params.rc < 0.5 * float(Ls.min()):
        # every pair has at most one image within rc: minimum image via a k-d tree
        tree = cKDTree(np.mod(pos, Ls), boxsize=Ls)
        chunk = 4096
        for t0 in range(0, tgt.shape[0], chunk):
            ti = tgt[t0:t0 + chunk]
            lists = tree.query_ball_point(np.mod(pos[ti], Ls), params.rc)
            ii = np.concatenate([np.full(len(l), n) for n, l in enumerate(lists)]).astype(np.int64)
            jj = np.concatenate([np.asarray(l, dtype=np.int64) for l in lists])
            sel = jj != ti[ii]
            ii, jj = ii[sel], jj[sel]
            if ii.size == 0:
                continue
            dv = pos[ti[ii]] - pos[jj]
            dv -= Ls * np.round(dv / Ls)
            for c0 in range(0, ii.size, 200000):
                accumulate(t0, ii[c0:c0 + 200000], jj[c0:c0 + 200000], dv[c0:c0 + 200000])
        return out
    chunk = max(1, 20000 // max(1, shifts.shape[0]))
    for t0 in range(0, tgt.shape[0], chunk):
        ti = tgt[t0:t0 + chunk]
        d0 = pos[ti][:, None, :] - pos[None, :, :]                # [t, N, 3]
        s = d0 @ inv.T
        d0 = (s - np.round(s)) @ box.T                            # minimum image
        d = d0[:, :, None, :] + shifts[None, None, :, :]          # [t, N, S, 3]
        r = np.linalg.norm(d, axis=-1)
        keep = (r < params.rc) & (r > 0.0)
        ii, jj, ss = np.nonzero(keep)
        if ii.size == 0:
            continue
        accumulate(t0, ii, jj, d[ii, jj, ss])
    return out


def wave_part(pos, rad, box, x, params: EwaldParams, targets=None, kblock: int | None = None) -> np.ndarray:
    """(1/V) sum over the k-set of exp(-i k.r_i) K(k) sum_j exp(i k.r_j) x_j,
    including j = i (the wave-space self term is removed in self_part)."""
    N = pos.shape[0]
    tgt = np.arange(N) if targets is None else np.asarray(targets)
    if kblock is None:  # keep the [N, kblock] phase arrays near 2e7 entries
        kblock = int(max(16, min(4096, 2e7 // max(N, 1))))
    V = abs(np.linalg.det(box))
    syms = block_symbols(params.eta)
    kv = k_vectors(box, params)
    out = np.zeros((tgt.shape[0], 12, x.shape[2]), dtype=np.complex128)
    Aj = rad ** 2
    Ai = rad[tgt] ** 2
    xq = np.stack([x, Aj[:, None, None] * x], axis=1).astype(np.complex128)   # [N, q, b, c]
    for k0 in range(0, kv.shape[0], kblock):
        k = kv[k0:k0 + kblock]
        k2 = np.einsum("ij,ij->i", k, k)
        ph_src = np.exp(1j * (pos @ k.T))                           # [N, K]
        S = np.einsum("nk,nqbc->kqbc", ph_src, xq, optimize=True)  # structure sums
        ph_tgt = np.exp(-1j * (pos[tgt] @ k.T))                     # [T, K]
        for fam in ("stokes", "laplace"):
            alphas, C = syms[fam]
            mono = np.prod(k[:, None, :] ** alphas[None, :, :], axis=-1)          # [K, A]
            Kpq = np.einsum("ka,apqij->kpqij", mono, C, optimize=True)            # [K, p, q, 12, 12]
            Kpq *= _wave_kernel(fam, k2, params.xi)[:, None, None, None, None]
            G = np.einsum("kpqab,kqbc->kpac", Kpq, S, optimize=True)              # [K, p, a, c]
            out += np.einsum("tk,kac->tac", ph_tgt, G[:, 0], optimize=True)
            out += Ai[:, None, None] * np.einsum("tk,kac->tac", ph_tgt, G[:, 1], optimize=True)
    assert np.max(np.abs(out.imag)) <= 1e-9 * max(1.0, np.max(np.abs(out.real)))
    return out.real / V


def _angular_moment(a: int, b: int, c: int) -> float:
    """Integral over the unit sphere of khat_x^a khat_y^b khat_z^c."""
    if a % 2 or b % 2 or c % 2:
        return 0.0

    def dfact(n):
        return 1.0 if n <= 0 else float(np.prod(np.arange(n, 0, -2)))
    return 4.0 * math.pi * dfact(a - 1) * dfact(b - 1) * dfact(c - 1) / dfact(a + b + c + 1)


def wave_self_block(a: float, xi: float, eta: float = 1.0) -> np.ndarray:
    """Continuum integral d^3k/(2pi)^3 of the i=j wave-space block, i.e. the
    part of the wave sum that belongs to the sphere's own (non-periodic)
    singular field (eq. uf-self and its analogues for the other blocks)."""
    syms = block_symbols(eta)
    A = a * a
    W = np.zeros((12, 12), dtype=np.complex128)
    for fam in ("stokes", "laplace"):
        alphas, C = syms[fam]
        Cs = C[:, 0, 0] + A * (C[:, 1, 0] + C[:, 0, 1]) + A * A * C[:, 1, 1]
        for n, (p, q, r) in enumerate(alphas):
            ang = _angular_moment(p, q, r)
            if ang == 0.0:
                continue
            deg = p + q + r
            if fam == "stokes":
                # int_0^inf k^(deg+2) (1 + k^2/4xi^2) e^{-k^2/4xi^2} / k^4 dk
                pw = deg - 2
                rad = _gauss_moment(pw, xi) + _gauss_moment(pw + 2, xi) / (4 * xi * xi)
            else:
                rad = _gauss_moment(deg, xi)
            W += Cs[n] * ang * rad / (2.0 * math.pi) ** 3
    assert np.max(np.abs(W.imag)) < 1e-12
    return W.real


def _gauss_moment(p: int, xi: float) -> float:
    """int_0^inf k^p exp(-k^2/(4 xi^2)) dk."""
    return 0.5 * (2.0 * xi) ** (p + 1) * gamma((p + 1) / 2.0)


def self_part(rad, x, params: EwaldParams, targets=None) -> np.ndarray:
    """Single-sphere mobility minus the wave-space self block, per target."""
    tgt = np.arange(rad.shape[0]) if targets is None else np.asarray(targets)
    out = np.zeros((tgt.shape[0], 12, x.shape[2]))
    cache = {}
    for n, i in enumerate(tgt):
        a = float(rad[i])
        if a not in cache:
            ws = wave_self_block(a, params.xi, params.eta)
            cache[a] = self_mobility(a, params.eta) - ws
        out[n] = cache[a] @ x[i]
    return out


# ---------------------------------------------------------------------------
# public entry points

def apply(pos, rad, box, x, params: EwaldParams | None = None, targets=None) -> np.ndarray:
    """y = M x for x of shape [N, 12] or [N, 12, C]; returns the same layout
    (restricted to `targets` when given). params=None: converged sum."""
    pos = np.asarray(pos, dtype=np.float64)
    rad = np.asarray(rad, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    squeeze = x.ndim == 2
    X = x[:, :, None] if squeeze else x
    if params is None:
        params = converged_params(box, rad)
    tgt = np.arange(pos.shape[0]) if targets is None else np.asarray(targets)
    y = np.zeros((tgt.shape[0], 12, X.shape[2]))
    if params.parts & PARTS_REAL:
        y += real_part(pos, rad, box, X, params, targets)
    if params.parts & PARTS_WAVE:
        y += wave_part(pos, rad, box, X, params, targets)
    if params.parts & PARTS_SELF:
        y += self_part(rad, X, params, targets)
    return y[:, :, 0] if squeeze else y


def dense_matrix(pos, rad, box, params: EwaldParams | None = None) -> np.ndarray:
    """The 12N x 12N matrix of M (small N only)."""
    N = pos.shape[0]
    E = np.eye(12 * N).reshape(N, 12, 12 * N)
    return apply(pos, rad, box, E, params).reshape(12 * N, 12 * N)


def pair_block_real(d, ai: float, aj: float, xi: float, eta: float = 1.0) -> np.ndarray:
    """The real-space 12x12 block for one displacement d = r_i - r_j (no images).
    With xi = 0 this is the free-space (unbounded fluid) coupling."""
    d = np.asarray(d, dtype=np.float64).reshape(1, 3)
    r = np.linalg.norm(d, axis=1)
    syms = block_symbols(eta)
    out = np.zeros((12, 12))
    for fam in ("stokes", "laplace"):
        alphas, C = syms[fam]
        Cr = (C * (1j) ** alphas.sum(1)[:, None, None, None, None]).real
        Cs = Cr[:, 0, 0] + ai * ai * Cr[:, 1, 0] + aj * aj * Cr[:, 0, 1] + ai * ai * aj * aj * Cr[:, 1, 1]
        fh = hierarchy(fam, r, xi, int(alphas.sum(1).max()))
        D = radial_derivatives(d, fh, alphas)[0]
        out += np.einsum("n,nab->ab", D, Cs)
    return out
