"""Seeded synthetic suspensions: positions, radii, boxes and force-moment inputs.

This module only draws inputs. It holds none of the mobility arithmetic, so the
oracle and the GPU path can both be fed from it without sharing any of the
method's code.

Placement follows the paper's workloads (random hard-sphere suspensions in a
periodic cube, monodisperse or bidisperse, Sec. 5.1 and Sec. 6): spheres are
dropped uniformly at a reduced radius and then inflated in steps; after each
step overlapping pairs are pushed apart until no pair overlaps. The result is a
random, non-overlapping configuration. It is not an equilibrium hard-sphere
ensemble (the paper's Lubachevsky-Stillinger packings are not reproduced).

Force moments use the 12-component layout (F3, T3, five traceless stresslet
coordinates, trace coordinate) and are drawn i.i.d. N(0, 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.spatial import cKDTree


@dataclass
class Suspension:
    pos: np.ndarray      # [N, 3] float64, inside [0, L)^3
    radius: np.ndarray   # [N] float64
    box: np.ndarray      # [3, 3] float64, columns are the lattice vectors
    phi: float           # achieved volume fraction
    min_gap: float       # min over pairs of r_ij / (a_i + a_j) - 1 (inf if N < 2)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def L(self) -> float:
        return float(self.box[0, 0])


def box_length(radius: np.ndarray, phi: float) -> float:
    """Cube edge L such that sum(4/3 pi a^3) / L^3 = phi."""
    vol = float(np.sum(4.0 / 3.0 * math.pi * radius ** 3))
    return (vol / phi) ** (1.0 / 3.0)


def _pairs_overlapping(pos, rad, L, margin):
    tree = cKDTree(pos, boxsize=L)
    rmax = 2.0 * float(rad.max()) * (1.0 + margin)
    pairs = tree.query_pairs(rmax, output_type="ndarray")
    if pairs.size == 0:
        return pairs, np.zeros((0, 3)), np.zeros(0)
    d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
    d -= L * np.round(d / L)
    r = np.sqrt(np.einsum("ij,ij->i", d, d))
    need = (rad[pairs[:, 0]] + rad[pairs[:, 1]]) * (1.0 + margin)
    sel = r < need
    return pairs[sel], d[sel], (need[sel] - r[sel])


def place_spheres(radius: np.ndarray, L: float, rng: np.random.Generator,
                  margin: float = 1e-3, max_sweeps: int = 20000) -> np.ndarray:
    """Random non-overlapping placement of spheres with the given radii in a
    periodic cube of edge L. Every pair ends with r_ij >= (a_i + a_j)(1 + margin/2).

    Overlaps are relaxed on a Verlet pair list (cut-off 2 a_max + skin) that is
    rebuilt once any sphere has moved more than half the skin."""
    n = radius.shape[0]
    pos = rng.uniform(0.0, L, size=(n, 3))
    if n < 2:
        return pos
    skin = 0.3 * float(radius.max())
    scales = [0.6, 0.75, 0.85, 0.92, 0.97, 1.0]
    for s in scales:
        rad = radius * s
        pairs = None
        ref = None
        for _ in range(max_sweeps):
            if pairs is None or np.max(np.abs(((pos - ref + 0.5 * L) % L) - 0.5 * L)) > 0.5 * skin:
                tree = cKDTree(pos, boxsize=L)
                pairs = tree.query_pairs(2.0 * float(rad.max()) * (1.0 + margin) + skin,
                                         output_type="ndarray")
                ref = pos.copy()
            if pairs.shape[0] == 0:
                break
            d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
            d -= L * np.round(d / L)
            r = np.sqrt(np.einsum("ij,ij->i", d, d))
            need = (rad[pairs[:, 0]] + rad[pairs[:, 1]]) * (1.0 + margin)
            sel = r < need
            if not np.any(sel):
                break
            u = d[sel] / np.maximum(r[sel], 1e-12)[:, None]
            # a small absolute extra step keeps round-off-sized overlaps from stalling
            dp = u * (0.55 * (need[sel] - r[sel]) + 0.05 * margin * need[sel])[:, None]
            np.add.at(pos, pairs[sel, 0], dp)
            np.add.at(pos, pairs[sel, 1], -dp)
            pos %= L
        else:
            raise RuntimeError("placement did not converge; lower phi or raise max_sweeps")
    pairs, _, _ = _pairs_overlapping(pos, radius, L, 0.5 * margin)
    if pairs.shape[0]:
        raise RuntimeError("placement left overlapping pairs")
    return pos


def min_gap(pos, radius, L) -> float:
    n = pos.shape[0]
    if n < 2:
        return math.inf
    tree = cKDTree(pos, boxsize=L)
    pairs = tree.query_pairs(2.0 * float(radius.max()) * 1.5, output_type="ndarray")
    if pairs.size == 0:
        return math.inf
    d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
    d -= L * np.round(d / L)
    r = np.sqrt(np.einsum("ij,ij->i", d, d))
    return float(np.min(r / (radius[pairs[:, 0]] + radius[pairs[:, 1]]) - 1.0))


def cube(L: float) -> np.ndarray:
    return np.eye(3) * L


def make_suspension(radius: np.ndarray, phi: float, seed: int) -> Suspension:
    rng = np.random.Generator(np.random.PCG64(seed))
    L = box_length(radius, phi)
    pos = place_spheres(radius, L, rng)
    return Suspension(pos=pos, radius=radius.astype(np.float64), box=cube(L),
                      phi=phi, min_gap=min_gap(pos, radius, L))


def in_cell(s: Suspension, box: np.ndarray, margin: float = 1e-3, max_sweeps: int = 5000) -> Suspension:
    """The same spheres moved as little as needed to be non-overlapping in
    another periodic cell of the same volume (columns of box are the lattice
    vectors, e.g. the sheared cell a2 = (gamma L, L, 0)): a cube configuration
    can overlap through the images of a sheared lattice. Pairs are found by
    brute force over the 27 nearest lattice images (small suspensions only)
    and pushed apart along their separation until every pair has
    r_ij >= (a_i + a_j)(1 + margin/2)."""
    box = np.asarray(box, dtype=np.float64)
    inv = np.linalg.inv(box)
    rad = s.radius
    n = s.n
    if n > 4000:
        raise ValueError("in_cell is meant for small suspensions")
    shifts = np.array([(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)], dtype=np.float64)
    t = (s.pos @ inv.T) % 1.0
    need_all = (rad[:, None] + rad[None, :]) * (1.0 + margin)
    iu = np.triu_indices(n, 1)
    for _ in range(max_sweeps):
        pos = t @ box.T
        dt = t[:, None, :] - t[None, :, :]
        dt -= np.round(dt)
        d = (dt[:, :, None, :] + shifts[None, None, :, :]) @ box.T          # [n, n, 27, 3]
        r = np.linalg.norm(d, axis=-1)
        k = np.argmin(r, axis=2)
        rmin = np.take_along_axis(r, k[:, :, None], axis=2)[:, :, 0]
        sel = rmin[iu] < need_all[iu]
        if not np.any(sel):
            break
        i, j = iu[0][sel], iu[1][sel]
        dv = d[i, j, k[i, j]]
        rr = np.maximum(rmin[i, j], 1e-12)
        dp = dv / rr[:, None] * (0.55 * (need_all[i, j] - rr) + 0.05 * margin * need_all[i, j])[:, None]
        np.add.at(pos, i, dp)
        np.add.at(pos, j, -dp)
        t = (pos @ inv.T) % 1.0
    else:
        raise RuntimeError("relaxation in the cell did not converge")
    pos = t @ box.T
    gap = float(np.min(rmin[iu] / (rad[iu[0]] + rad[iu[1]]) - 1.0)) if n > 1 else math.inf
    return Suspension(pos=pos, radius=rad.copy(), box=box.copy(), phi=s.phi, min_gap=gap)


def monodisperse(n: int, phi: float, seed: int, a: float = 1.0) -> Suspension:
    return make_suspension(np.full(n, a, dtype=np.float64), phi, seed)


def bidisperse(n: int, phi: float, seed: int, a1: float = 1.0, a2: float = 2.0,
               y2: float = 0.5) -> Suspension:
    """Bidisperse suspension with size ratio a2/a1 and species-2 volume share y2
    (the paper's composition variables lambda, phi, y2; Sec. 2.1).
    Number of large spheres: n2 = round(n * x2) with x2 from y2 and the size ratio."""
    lam3 = (a2 / a1) ** 3
    x2 = y2 / (y2 + (1.0 - y2) * lam3)
    n2 = int(round(n * x2))
    rad = np.concatenate([np.full(n - n2, a1), np.full(n2, a2)])
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    rng.shuffle(rad)
    return make_suspension(rad, phi, seed)


def lognormal(n: int, phi: float, seed: int, median: float = 1.0, sigma: float = 0.2) -> Suspension:
    rng = np.random.Generator(np.random.PCG64(seed + 104729))
    rad = median * np.exp(sigma * rng.standard_normal(n))
    return make_suspension(rad, phi, seed)


def batch_member(k: int, seed: int = 4000) -> Suspension:
    """Member k of the many-suspension workload: N log-uniform in [500, 8000],
    phi uniform in [0.1, 0.45], lognormal radii (median 1, sigma 0.2), each in
    its own cube."""
    rng = np.random.default_rng(seed + k)
    n = int(np.exp(rng.uniform(np.log(500), np.log(8000))))
    phi = float(rng.uniform(0.1, 0.45))
    return lognormal(n, phi, seed + 1000 + k)


def force_moments(n: int, seed: int, columns: int | None = None) -> np.ndarray:
    """x (or b) with 12 components per particle, i.i.d. N(0, 1), float64.
    Drawn from a stream independent of the placement stream."""
    rng = np.random.Generator(np.random.PCG64(seed * 2654435761 % (2 ** 63) + 12345))
    shape = (n, 12) if columns is None else (n, 12, columns)
    return rng.standard_normal(shape)


def unit_norm_moments(n: int, seed: int) -> np.ndarray:
    """Moments rescaled so that |F_i| = |T_i| = |S_i| = 1 per particle, the
    normalisation the paper uses for its accuracy studies (Sec. 5.1)."""
    x = force_moments(n, seed)
    x[:, 0:3] /= np.linalg.norm(x[:, 0:3], axis=1, keepdims=True)
    x[:, 3:6] /= np.linalg.norm(x[:, 3:6], axis=1, keepdims=True)
    x[:, 6:12] /= np.linalg.norm(x[:, 6:12], axis=1, keepdims=True)
    return x


# ---- the named workloads -------------------------------------------------------

def config_small(seed: int = 1000) -> Suspension:
    """N=100 monodisperse spheres (a=1) at phi=0.1."""
    return monodisperse(100, 0.1, seed)


def config_bidisperse_solve(seed: int = 2000, n: int = 10000) -> Suspension:
    """N=10,000 spheres at radii 1 and 2, equal volume fraction per species,
    total phi=0.3."""
    return bidisperse(n, 0.3, seed, 1.0, 2.0, y2=0.5)


def config_large(seed: int = 3000, n: int = 100000) -> Suspension:
    """N=100,000 monodisperse spheres at phi=0.4."""
    return monodisperse(n, 0.4, seed)
