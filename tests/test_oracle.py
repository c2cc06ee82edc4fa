"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is a closed form,
a value the paper prints, an independent numerical construction (finite
differences of the Oseen tensor), or an invariance the exact operator has.
"""
import math

import numpy as np
import pytest

from oracle import ewald, solve, symbols
from paper_1506_08481_amd import workloads as wl

HASIMOTO_SC = 2.837297  # Hasimoto's simple-cubic constant (1959), 7 digits


def _unit(n, comp):
    x = np.zeros((n, 12))
    x[0, comp] = 1.0
    return x


# ---------------------------------------------------------------------------
# sedimenting / rotating simple-cubic array (one sphere per periodic cell)

@pytest.mark.parametrize("L", [6.0, 10.0, 25.0])
def test_sc_array_translation_hasimoto(L, paper):
    box = np.eye(3) * L
    y = ewald.apply(np.zeros((1, 3)), np.array([1.0]), box, _unit(1, 0))
    ratio = y[0, 0] * 6.0 * math.pi            # U 6 pi eta a / F
    expect = 1.0 - HASIMOTO_SC / L + 4.0 * math.pi / 3.0 / L ** 3
    assert abs(ratio - expect) < 6e-7 / L       # the constant is known to 7 digits
    # transverse components and the other outputs vanish by cubic symmetry
    assert np.max(np.abs(np.delete(y[0], 0))) < 1e-14
    # the paper's 3-digit form of the same coefficient: 1.76 (phi/N)^(1/3)
    phi = 4.0 * math.pi / 3.0 / L ** 3
    coef = (1.0 - ratio + phi) / phi ** (1.0 / 3.0)
    assert abs(coef - paper("sc_self_mobility_phi_coefficient")) < 0.005


@pytest.mark.parametrize("L,a", [(6.0, 1.0), (12.0, 2.0)])
def test_sc_array_rotation(L, a):
    # image correction of the spin from the curl of the periodic Oseen tensor:
    # Omega 8 pi eta a^3 / T = 1 - (4 pi/3)(a/L)^3, exact at this level
    box = np.eye(3) * L
    y = ewald.apply(np.zeros((1, 3)), np.array([a]), box, _unit(1, 4))
    assert abs(y[0, 4] * 8.0 * math.pi * a ** 3 - (1.0 - 4.0 * math.pi / 3.0 * (a / L) ** 3)) < 1e-13


def test_sc_array_radius_scaling():
    # U 6 pi eta a / F depends on a/L only (length scaling of Stokes flow)
    r1 = ewald.apply(np.zeros((1, 3)), np.array([1.0]), np.eye(3) * 9.0, _unit(1, 2))[0, 2] * 6 * math.pi
    r2 = ewald.apply(np.zeros((1, 3)), np.array([2.0]), np.eye(3) * 18.0, _unit(1, 2))[0, 2] * 12 * math.pi
    assert abs(r1 - r2) < 1e-14


# ---------------------------------------------------------------------------
# the paper's printed self terms

def test_wave_self_uf_matches_printed_formula(paper):
    c0, c2, c4, den = (paper(k) for k in ("uf_self_c0", "uf_self_c2", "uf_self_c4", "uf_self_den"))
    for a, xi in [(1.0, 0.5), (2.0, 0.3), (1.3, 1.1)]:
        W = ewald.wave_self_block(a, xi)
        printed = xi * (c0 + c2 * a * a * xi * xi + c4 * a ** 4 * xi ** 4) / (den * math.pi ** 1.5)
        assert np.allclose(np.diag(W)[:3], printed, rtol=1e-14, atol=0)


def test_single_sphere_self_terms(paper):
    a = 1.7
    S = symbols.self_mobility(a)
    assert np.isclose(S[0, 0], 1 / (paper("self_force_den") * math.pi * a), rtol=1e-15)
    assert np.isclose(S[3, 3], 1 / (paper("self_torque_den") * math.pi * a ** 3), rtol=1e-15)
    assert np.isclose(S[6, 6], 1 / (paper("self_stresslet_den") * math.pi * a ** 3), rtol=1e-14)
    assert np.isclose(S[11, 11], 1 / (paper("self_pressure_moment_den") * math.pi * a ** 3), rtol=1e-14)


# ---------------------------------------------------------------------------
# free-space limits (xi = 0) of the real-space blocks

def _oseen(r):
    rn = np.linalg.norm(r)
    return (np.eye(3) + np.outer(r, r) / rn ** 2) / rn


def _fd_grad(f, r, h=1e-4):
    """Fourth-order central differences; returns array with a trailing axis for d/dr."""
    out = []
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        out.append((-f(r + 2 * e) + 8 * f(r + e) - 8 * f(r - e) + f(r - 2 * e)) / (12 * h))
    return np.stack(out, axis=-1)


def _stresslet_field(S):
    # velocity of a point stresslet pushed on the fluid: -(1/8 pi) K:S with
    # K_abc = (d_c J_ab + d_b J_ac)/2, J the Oseen tensor (eq. mul-expand)
    def v(r):
        dJ = _fd_grad(_oseen, r, 1e-3)                      # [a, b, c] = d_c J_ab
        K = 0.5 * (dJ + np.transpose(dJ, (0, 2, 1)))
        return -np.einsum("abc,bc->a", K, S) / (8 * math.pi)
    return v


def test_free_space_rpy_and_rotlet():
    rng = np.random.default_rng(3)
    for _ in range(4):
        d = rng.normal(size=3)
        d *= (2.5 + 3 * rng.random()) / np.linalg.norm(d)
        ai, aj = 0.5 + rng.random(), 0.5 + rng.random()
        B = ewald.pair_block_real(d, ai, aj, 0.0)
        r = np.linalg.norm(d)
        rr = np.outer(d, d) / r ** 2
        s = ai * ai + aj * aj
        rpy = ((1 + s / (3 * r * r)) * np.eye(3) + (1 - s / (r * r)) * rr) / (8 * math.pi * r)
        assert np.allclose(B[0:3, 0:3], rpy, rtol=1e-13, atol=1e-16)
        # U_i <- T_j: rotlet T x r/(8 pi r^3) with r = r_i - r_j
        T = rng.normal(size=3)
        assert np.allclose(B[0:3, 3:6] @ T, np.cross(T, d) / (8 * math.pi * r ** 3), rtol=1e-12, atol=1e-16)
        # Omega_i <- T_j: (3 rr - I) T / (16 pi r^3)
        assert np.allclose(B[3:6, 3:6], (3 * rr - np.eye(3)) / (16 * math.pi * r ** 3), rtol=1e-12, atol=1e-16)
        # Omega_i <- F_j: (1/2) curl of the Oseen velocity
        F = rng.normal(size=3)
        v = lambda q: _oseen(q) @ F / (8 * math.pi)
        g = _fd_grad(v, d, 1e-4)                            # g[a, c] = d_c v_a
        curl = np.array([g[2, 1] - g[1, 2], g[0, 2] - g[2, 0], g[1, 0] - g[0, 1]])
        assert np.allclose(B[3:6, 0:3] @ F, 0.5 * curl, rtol=1e-8, atol=1e-12)


def test_free_space_stresslet_and_strain_point_limit():
    Y = symbols.traceless_basis()
    rng = np.random.default_rng(4)
    for _ in range(3):
        d = rng.normal(size=3)
        d *= 3.0 / np.linalg.norm(d)
        B = ewald.pair_block_real(d, 0.0, 0.0, 0.0)
        s = rng.normal(size=5)
        S = np.einsum("m,mab->ab", s, Y)
        v = _stresslet_field(S)
        assert np.allclose(B[0:3, 6:11] @ s, v(d), rtol=1e-7, atol=1e-12)
        # strain at i of the stresslet field: symmetric gradient projected on Y
        g = _fd_grad(v, d, 1e-3)
        e = np.einsum("mab,ab->m", Y, 0.5 * (g + g.T))
        assert np.allclose(B[6:11, 6:11] @ s, e, rtol=1e-6, atol=1e-10)
        # strain at i of a point force (Oseen field)
        F = rng.normal(size=3)
        gF = _fd_grad(lambda q: _oseen(q) @ F / (8 * math.pi), d, 1e-4)
        assert np.allclose(B[6:11, 0:3] @ F, np.einsum("mab,ab->m", Y, 0.5 * (gF + gF.T)), rtol=1e-8, atol=1e-12)


def test_free_space_faxen_terms_of_stresslet():
    # U_i <- S_j with radii: (1 + ai^2 lap/6)(1 + aj^2 lap/10) applied to the
    # stresslet field; its Laplacian is taken by finite differences.
    Y = symbols.traceless_basis()
    rng = np.random.default_rng(5)
    d = rng.normal(size=3)
    d *= 3.5 / np.linalg.norm(d)
    ai, aj = 1.0, 1.5
    s = rng.normal(size=5)
    S = np.einsum("m,mab->ab", s, Y)
    v = _stresslet_field(S)
    h = 2e-2
    lap = sum((v(d + h * e) - 2 * v(d) + v(d - h * e)) / h ** 2 for e in np.eye(3))
    expect = v(d) + (ai * ai / 6 + aj * aj / 10) * lap
    B = ewald.pair_block_real(d, ai, aj, 0.0)
    assert np.allclose(B[0:3, 6:11] @ s, expect, rtol=2e-4, atol=1e-8)


def test_free_space_compressible_couplings(paper):
    rng = np.random.default_rng(6)
    Y = symbols.traceless_basis()
    d = rng.normal(size=3)
    d *= 2.7 / np.linalg.norm(d)
    r = np.linalg.norm(d)
    B = ewald.pair_block_real(d, 1.0, 1.3, 0.0)
    s6 = 0.7                                   # trace coordinate, S_trace = sqrt(3) s6
    # source flow of the pressure moment, S r / (16 pi eta r^3)
    assert np.allclose(B[0:3, 11] * s6, math.sqrt(3) * s6 * d / (paper("source_flow_den") * math.pi * r ** 3),
                       rtol=1e-12, atol=0)
    # pressure Faxen law: -E_trace = ... - (3/(4 eta)) p', e6 = -E_trace/sqrt(3)
    F = rng.normal(size=3)
    p = F @ d / (paper("pressure_force_den") * math.pi * r ** 3)
    assert np.isclose(B[11, 0:3] @ F, -math.sqrt(3) / 4 * p, rtol=1e-12)
    # pressure of a stresslet: -(1/4pi) grad(r/r^3) : S  (eq. pres-multi-expans)
    sv = rng.normal(size=5)
    S = np.einsum("m,mab->ab", sv, Y)
    gradP = _fd_grad(lambda q: q / np.linalg.norm(q) ** 3, d, 1e-4)
    pS = -np.einsum("ab,ab->", gradP, S) / (4 * math.pi)
    assert np.isclose(B[11, 6:11] @ sv, -math.sqrt(3) / 4 * pS, rtol=1e-8)
    # torques and other pressure moments carry no pressure; sources carry no spin
    assert np.allclose(B[11, 3:6], 0) and B[11, 11] == 0 and np.allclose(B[3:6, 11], 0)


# ---------------------------------------------------------------------------
# Ewald consistency, symmetry, positive definiteness, invariances

@pytest.fixture(scope="module")
def small_bidisperse():
    s = wl.bidisperse(10, 0.2, 21)
    return s, wl.force_moments(s.n, 9)


def test_xi_independence(small_bidisperse):
    s, x = small_bidisperse
    ys = [ewald.apply(s.pos, s.radius, s.box, x, ewald.converged_params(s.box, s.radius, xi=xi))
          for xi in (0.35, 0.6, 1.0)]
    for y in ys[1:]:
        assert np.linalg.norm(y - ys[0]) / np.linalg.norm(ys[0]) < 1e-13


def test_cutoffs_converged(small_bidisperse):
    s, x = small_bidisperse
    y8 = ewald.apply(s.pos, s.radius, s.box, x, ewald.converged_params(s.box, s.radius, xi=0.6, tol_exp=8.0))
    y11 = ewald.apply(s.pos, s.radius, s.box, x, ewald.converged_params(s.box, s.radius, xi=0.6, tol_exp=11.0))
    assert np.linalg.norm(y11 - y8) / np.linalg.norm(y11) < 1e-15


def test_split_parts_add_up(small_bidisperse):
    s, x = small_bidisperse
    p = ewald.converged_params(s.box, s.radius, xi=0.7)
    full = ewald.apply(s.pos, s.radius, s.box, x, p)
    acc = 0
    for parts in (ewald.PARTS_REAL, ewald.PARTS_WAVE, ewald.PARTS_SELF):
        q = ewald.EwaldParams(xi=p.xi, rc=p.rc, kc=p.kc, parts=parts)
        acc = acc + ewald.apply(s.pos, s.radius, s.box, x, q)
    assert np.allclose(acc, full, rtol=0, atol=1e-14 * np.abs(full).max())


@pytest.fixture(scope="module")
def dense8():
    s = wl.bidisperse(8, 0.25, 31)
    M = ewald.dense_matrix(s.pos, s.radius, s.box, ewald.converged_params(s.box, s.radius, xi=0.8))
    return s, M


def test_symmetry_and_positive_definiteness(dense8):
    s, M = dense8
    n = s.n
    A = M.reshape(n, 12, n, 12)[:, :11, :, :11].reshape(11 * n, 11 * n)
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


def test_pressure_moment_one_way_coupling(dense8):
    s, M = dense8
    n = s.n
    B = M.reshape(n, 12, n, 12)
    for i in range(n):
        for j in range(n):
            assert np.allclose(B[i, 11, j, 3:6], 0, atol=1e-15)        # no pressure from torques
            if i != j:
                assert abs(B[i, 11, j, 11]) < 1e-15                    # sources make no pressure


def test_dense_solve_recovers_rhs(dense8):
    s, M = dense8
    b = wl.force_moments(s.n, 77)
    x = solve.dense_solve(s.pos, s.radius, s.box, b, ewald.converged_params(s.box, s.radius, xi=0.8))
    assert np.linalg.norm(M @ x.ravel() - b.ravel()) < 1e-11 * np.linalg.norm(b)


def _rot_z90():
    return np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])


def _rotate_moments(x, R):
    Y = symbols.traceless_basis()
    out = x.copy()
    out[:, 0:3] = x[:, 0:3] @ R.T
    out[:, 3:6] = x[:, 3:6] @ R.T          # proper rotation: pseudovectors rotate alike
    S = np.einsum("nm,mab->nab", x[:, 6:11], Y)
    S = np.einsum("ac,ncd,bd->nab", R, S, R)
    out[:, 6:11] = np.einsum("mab,nab->nm", Y, S)
    return out


def test_invariances(small_bidisperse):
    s, x = small_bidisperse
    p = ewald.converged_params(s.box, s.radius, xi=0.6)
    y = ewald.apply(s.pos, s.radius, s.box, x, p)
    # translation and periodic shift of one sphere
    shift = np.array([0.37, -1.2, 2.9])
    pos2 = s.pos + shift
    pos2[3] += s.box[:, 1]
    assert np.allclose(ewald.apply(pos2, s.radius, s.box, x, p), y, rtol=0, atol=1e-13 * np.abs(y).max())
    # permutation
    perm = np.random.default_rng(1).permutation(s.n)
    yp = ewald.apply(s.pos[perm], s.radius[perm], s.box, x[perm], p)
    assert np.allclose(yp, y[perm], rtol=0, atol=1e-13 * np.abs(y).max())
    # 90 degree rotation about z of the whole cubic cell
    R = _rot_z90()
    yr = ewald.apply(s.pos @ R.T, s.radius, s.box, _rotate_moments(x, R), p)
    assert np.allclose(yr, _rotate_moments(y, R), rtol=0, atol=1e-13 * np.abs(y).max())


def test_periodic_strain_row_is_the_gradient_of_the_velocity_row():
    """With a vanishing target radius the Faxen laws of the target reduce to
    point values (Sec. 2.2: eqs. faxen-f, faxen-t, faxen-s), so in the
    periodic sum the strain output of any source moment is the symmetric
    gradient of the velocity output with respect to the target position, and
    the spin output half its curl. Checked by
    fourth-order finite differences of the full Ewald sum in a box of edge 8,
    where the periodic images carry 22-43 % of these couplings: the image
    parts of E<-F, E<-S (whose velocity rows Hasimoto's array and the
    symmetry M_US = M_EF^T fix) and E<-trace are pinned in absolute size."""
    import dataclasses
    Y = symbols.traceless_basis()
    aj = 1.5                               # source Faxen terms present
    box = np.eye(3) * 8.0
    d = np.array([2.1, -1.3, 2.6])
    rad = np.array([0.0, aj])
    p = ewald.converged_params(box, np.array([1.0, aj]), xi=0.6)
    # the target carries no moments: its self part (1/a terms) is left out
    p = dataclasses.replace(p, parts=ewald.PARTS_REAL | ewald.PARTS_WAVE)
    x = np.zeros((2, 12, 12))
    x[1] = np.eye(12)                      # every moment of the source, one per column

    def y(q):
        return ewald.apply(np.stack([q, np.zeros(3)]), rad, box, x, p, targets=np.array([0]))[0]

    h = 5e-3
    g = np.zeros((3, 3, 12))               # g[b, a, c] = d U_b / d q_a for source column c
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        g[:, a, :] = (-y(d + 2 * e)[0:3] + 8 * y(d + e)[0:3] - 8 * y(d - e)[0:3] + y(d - 2 * e)[0:3]) / (12 * h)
    strain = np.einsum("mab,abc->mc", Y, 0.5 * (g + g.transpose(1, 0, 2)))
    y0 = y(d)
    # the spin read-out is half the curl of the velocity (eq. faxen-t)
    curl = np.stack([g[2, 1] - g[1, 2], g[0, 2] - g[2, 0], g[1, 0] - g[0, 1]])
    assert np.linalg.norm(y0[3:6] - 0.5 * curl) < 1e-9 * np.linalg.norm(0.5 * curl)
    E = y0[6:11]
    for cols in (slice(0, 3), slice(6, 11), slice(11, 12)):
        ref = strain[:, cols]
        assert np.linalg.norm(E[:, cols] - ref) < 1e-9 * np.linalg.norm(ref)
        # a flipped sign or a dropped image sum fails by far more than the bound
        free = ewald.pair_block_real(d, 0.0, aj, 0.0)[6:11, cols]
        assert np.linalg.norm(free - ref) > 0.2 * np.linalg.norm(ref)


def test_periodic_source_flow_identities():
    """The velocity of a pressure-moment source (Sec. 2.3: a point source of
    fluid, a potential flow) summed over the periodic images, with the k = 0
    mode left out, is curl-free and has divergence -kappa / (4 eta V) away
    from the source (the uniform sink that keeps the cell's volume fixed),
    kappa the source strength of the free-space closed form; by the point
    symmetry of the lattice it vanishes at the half-lattice points. Checked
    with fourth-order finite differences of the full sum at a point target:
    this fixes the image part of the velocity of a pressure moment (and
    through the gradient relation of the strain row, of E<-trace)."""
    import dataclasses
    L, aj = 8.0, 1.0
    box = np.eye(3) * L
    rad = np.array([0.0, aj])
    p = ewald.converged_params(box, np.array([1.0, aj]), xi=0.6)
    p = dataclasses.replace(p, parts=ewald.PARTS_REAL | ewald.PARTS_WAVE)
    x = np.zeros((2, 12))
    x[1, 11] = 1.0

    def u(q):
        return ewald.apply(np.stack([q, np.zeros(3)]), rad, box, x, p, targets=np.array([0]))[0][0:3]

    d0 = np.array([2.1, -1.3, 2.6])
    free = ewald.pair_block_real(d0, 0.0, aj, 0.0)[0:3, 11]     # kappa d / (16 pi eta |d|^3)
    kappa = float(free @ d0) * 16.0 * math.pi * np.linalg.norm(d0) ** 3 / float(d0 @ d0)
    assert abs(kappa - math.sqrt(3.0)) < 1e-12   # trace coordinate s6 = tr(S)/sqrt(3)
    for d in (d0, np.array([-3.0, 0.7, 1.1])):
        h = 5e-3
        g = np.zeros((3, 3))
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            g[:, a] = (-u(d + 2 * e) + 8 * u(d + e) - 8 * u(d - e) + u(d - 2 * e)) / (12 * h)
        div = -kappa / (4.0 * L ** 3)
        assert abs(np.trace(g) - div) < 1e-8 * abs(div)
        assert np.linalg.norm(g - g.T) < 1e-9 * np.linalg.norm(g)
    for d in ([L / 2, 0, 0], [0, L / 2, 0], [L / 2, L / 2, 0], [L / 2, L / 2, L / 2]):
        assert np.linalg.norm(u(np.array(d, dtype=float))) < 1e-12 * np.linalg.norm(free)


def test_periodic_pressure_readout_obeys_stokes():
    """The trace output row at a point target reads out the disturbance
    pressure (pressure Faxen law, eq. faxen-p; the factor c is that of the
    free-space closed form). Away from the sources the periodic fields obey
    Stokes' equations, grad p = eta lap u - F / V for a force (the uniform
    pressure gradient that carries the dropped k = 0 force) and grad p =
    eta lap u for torques and stresslets. Checked with fourth-order finite
    differences of the full sum (first derivatives of the pressure row,
    second of the velocity row): this fixes the image part of the trace
    output row of force, torque and stresslet sources through the velocity
    rows."""
    import dataclasses
    L, aj = 8.0, 1.5
    box = np.eye(3) * L
    rad = np.array([0.0, aj])
    p = ewald.converged_params(box, np.array([1.0, aj]), xi=0.6)
    p = dataclasses.replace(p, parts=ewald.PARTS_REAL | ewald.PARTS_WAVE)
    x = np.zeros((2, 12, 11))
    x[1, :11] = np.eye(11)                 # force, torque and stresslet sources

    def y(q):
        return ewald.apply(np.stack([q, np.zeros(3)]), rad, box, x, p, targets=np.array([0]))[0]

    d = np.array([2.1, -1.3, 2.6])
    free = ewald.pair_block_real(d, 0.0, aj, 0.0)
    c = float(free[11, 0:3] @ d) * 4.0 * math.pi * np.linalg.norm(d) ** 3 / float(d @ d)   # e6 = c p
    y0 = y(d)
    gp = np.zeros((3, 11))
    lap = np.zeros((3, 11))
    for a in range(3):
        e = np.zeros(3)
        e[a] = 5e-3
        gp[a] = (-y(d + 2 * e)[11] + 8 * y(d + e)[11] - 8 * y(d - e)[11] + y(d - 2 * e)[11]) / (12 * 5e-3) / c
        e[a] = 2e-2
        lap += (-y(d + 2 * e)[0:3] + 16 * y(d + e)[0:3] - 30 * y0[0:3] + 16 * y(d - e)[0:3]
                - y(d - 2 * e)[0:3]) / (12 * 2e-2 ** 2)
    rhs = lap.copy()
    rhs[:, 0:3] -= np.eye(3) / L ** 3
    for cols in (slice(0, 3), slice(3, 11)):
        assert np.linalg.norm(gp[:, cols] - rhs[:, cols]) < 1e-7 * np.linalg.norm(gp[:, cols])
    # the background term is not negligible: its sign flipped misses by far
    assert np.linalg.norm(gp[:, 0:3] - lap[:, 0:3] - np.eye(3) / L ** 3) > 0.5 * np.linalg.norm(gp[:, 0:3])


def test_pair_image_correction_tends_to_hasimoto():
    # two spheres close together in a large box: the periodic coupling differs
    # from the free-space one by the self-image constant, -2.837297/(6 pi eta L)
    for L in (30.0, 60.0):
        d = np.array([1.3, -2.1, 0.8])
        pos = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0] - d])
        rad = np.array([1.0, 1.0])
        M = ewald.dense_matrix(pos, rad, np.eye(3) * L).reshape(2, 12, 2, 12)
        diff = M[0, 0:3, 1, 0:3] - ewald.pair_block_real(d, 1.0, 1.0, 0.0)[0:3, 0:3]
        corr = -HASIMOTO_SC / (6 * math.pi * L)
        # remaining terms are O(r^2/L^3)
        assert np.allclose(diff, corr * np.eye(3), rtol=0, atol=60.0 / L ** 3)


def test_one_way_solve_satisfies_its_equations(dense8):
    # f solves the incompressible rows with only the self part of the pressure
    # moments as sources; the trace rows then hold exactly (pressure Faxen law)
    s, M = dense8
    n = s.n
    B = M.reshape(n, 12, n, 12)
    b = wl.force_moments(n, 5)
    x = solve.one_way_solve(s.pos, s.radius, s.box, b, ewald.converged_params(s.box, s.radius, xi=0.8))
    y = (M @ x.reshape(-1)).reshape(n, 12)
    assert np.allclose(y[:, 11], b[:, 11], rtol=0, atol=1e-12)          # trace rows exact
    m_self = np.array([B[i, 11, i, 11] for i in range(n)])
    s_int = x[:, 11] - b[:, 11] / m_self                                # interaction part
    feedback = np.einsum("iajb,jb->ia", B[:, :11, :, 11:12], s_int[:, None])
    assert np.allclose(y[:, :11] - feedback, b[:, :11], rtol=0, atol=1e-11)


# ---------------------------------------------------------------------------
# the split-diagnostic wave sum over the grid's k-set (|q_d| < M/2)

def test_grid_kset_is_the_grid_without_nyquist_planes():
    # the k-set of an M^3 grid: every integer q with |q_d| < M/2 except q = 0,
    # symmetric under q -> -q, mapped by k = B q (the cube: k = 2 pi q / L)
    L = 7.0
    for M in (8, 16):
        k = ewald.k_vectors(np.eye(3) * L, ewald.EwaldParams(xi=0.5, rc=1.0, grid=(M, M, M)))
        q = np.rint(k * L / (2 * np.pi)).astype(int)
        assert np.allclose(q * 2 * np.pi / L, k, atol=1e-12)
        assert k.shape[0] == (M - 1) ** 3 - 1
        assert np.abs(q).max() == M // 2 - 1
        keys = {tuple(v) for v in q}
        assert all(tuple(-v) in keys for v in q) and (0, 0, 0) not in keys


def test_grid_kset_wave_sum_converges_to_the_converged_wave_sum(small_bidisperse):
    # once the grid's Nyquist wavenumber pi M / L lies far beyond the
    # converged cut-off, the grid k-set sum equals the converged wave sum
    s, x = small_bidisperse
    conv = ewald.converged_params(s.box, s.radius, xi=0.6, tol_exp=6.5)
    yk = ewald.apply(s.pos, s.radius, s.box, x, ewald.EwaldParams(xi=0.6, rc=conv.rc, kc=conv.kc,
                                                                   parts=ewald.PARTS_WAVE))
    M = int(2 * np.ceil(conv.kc * s.L / (2 * np.pi))) + 4
    yg = ewald.apply(s.pos, s.radius, s.box, x, ewald.EwaldParams(xi=0.6, rc=conv.rc, grid=(M, M, M),
                                                                   parts=ewald.PARTS_WAVE))
    assert np.linalg.norm(yg - yk) / np.linalg.norm(yk) < 1e-13
    # a coarse grid truncates the sum visibly
    yc = ewald.apply(s.pos, s.radius, s.box, x, ewald.EwaldParams(xi=0.6, rc=conv.rc, grid=(6, 6, 6),
                                                                   parts=ewald.PARTS_WAVE))
    assert np.linalg.norm(yc - yk) / np.linalg.norm(yk) > 1e-6
