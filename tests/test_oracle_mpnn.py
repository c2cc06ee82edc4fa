"""Pins of the reference network of the learned preconditioner (oracle/mpnn.py)
against things other than itself: finite differences, rotation covariance,
the span of the free-space pair mobility, permutation invariance, and the
special case that reduces to the block-diagonal preconditioner."""
import numpy as np
import pytest

from oracle import ewald, mpnn
from oracle.symbols import traceless_basis


def _system(seed=0, n=10, L=8.0):
    rng = np.random.default_rng(seed)
    rad = np.where(rng.random(n) < 0.5, 1.0, 1.5)
    # non-overlapping random placement by rejection
    pos = np.zeros((n, 3))
    k = 0
    while k < n:
        p = rng.uniform(0, L, 3)
        d = pos[:k] - p
        d -= L * np.round(d / L)
        if k == 0 or np.all(np.linalg.norm(d, axis=1) > rad[:k] + rad[k] + 0.05):
            pos[k] = p
            k += 1
    return pos, rad


def _iso_blocks(rad):
    B = np.zeros((len(rad), 12, 12))
    for i, a in enumerate(rad):
        d = [6 * np.pi * a] * 3 + [8 * np.pi * a ** 3] * 3 + [20 / 3 * np.pi * a ** 3] * 5 + [1.0]
        B[i] = np.diag(d)
    return B


def _aniso_blocks(rad, seed):
    rng = np.random.default_rng(seed)
    B = _iso_blocks(rad)
    for i in range(len(rad)):
        G = 0.2 * rng.standard_normal((12, 12)) * np.sqrt(np.outer(np.diag(B[i]), np.diag(B[i])))
        B[i] = B[i] + G @ G.T / 12
    return B


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -7), 3.0e38, 1 + 2 ** -8 + 2 ** -20])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, -(1 + 2 ** -7), (1 + 98 / 128) * 2.0 ** 127, 1 + 2 ** -7])
    np.testing.assert_allclose(mpnn.bf16(x), want, rtol=1e-7)


def test_gradient_matches_finite_differences():
    pos, rad = _system(1)
    L = 8.0
    theta = mpnn.init_params(3, head_scale=0.3)
    rng = np.random.default_rng(5)
    p = mpnn.unpack(theta)   # biases start at zero: give them values
    for name in p:
        if name.startswith("b_"):
            p[name] = 0.1 * rng.standard_normal(p[name].shape)
    theta = mpnn.pack(p)
    B = _aniso_blocks(rad, 7)
    b = rng.standard_normal((2, len(rad), 12))
    xs = rng.standard_normal((2, len(rad), 12)) * np.sqrt(np.einsum("ncc->nc", B))[None] * 3
    loss, grad, _ = mpnn.loss_grad(theta, pos, rad, L, B, b, xs, bf=False)
    assert loss > 0
    off = 0
    for name, shape in mpnn.layout():
        size = int(np.prod(shape))
        d = np.zeros_like(theta)
        d[off:off + size] = rng.standard_normal(size)
        off += size
        eps = 1e-6
        lp = mpnn.loss_grad(theta + eps * d, pos, rad, L, B, b, xs, bf=False)[0]
        lm = mpnn.loss_grad(theta - eps * d, pos, rad, L, B, b, xs, bf=False)[0]
        fd = (lp - lm) / (2 * eps)
        an = grad @ d
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * loss), (name, fd, an)


def test_residual_loss_gradient_matches_finite_differences():
    pos, rad = _system(6)
    n = len(rad)
    rng = np.random.default_rng(8)
    G = rng.standard_normal((11 * n, 11 * n))
    Amat = G @ G.T / (11 * n) + np.eye(11 * n)

    def Aop(v):
        return (Amat @ v[:, :11].reshape(-1)).reshape(n, 11)

    theta = mpnn.init_params(5, head_scale=0.3)
    B = _aniso_blocks(rad, 9)
    b = rng.standard_normal((2, n, 12))
    loss, grad, x0 = mpnn.residual_loss_grad(theta, pos, rad, 8.0, B, b, Aop, bf=False)
    # the loss is what it says
    want = np.mean([np.sum((b[q, :, :11] - Aop(x0[q])) ** 2) / np.sum(b[q, :, :11] ** 2) for q in range(2)])
    assert abs(loss - want) < 1e-12 * want
    for k in range(4):
        d = rng.standard_normal(theta.size)
        eps = 1e-6
        lp = mpnn.residual_loss_grad(theta + eps * d, pos, rad, 8.0, B, b, Aop, bf=False)[0]
        lm = mpnn.residual_loss_grad(theta - eps * d, pos, rad, 8.0, B, b, Aop, bf=False)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grad @ d) <= 1e-6 * max(abs(grad @ d), 1e-3 * loss)


def _rep(R):
    """11x11 action of rotation R on (F, T, S-coordinates)."""
    Y = traceless_basis()
    D = np.zeros((11, 11))
    D[:3, :3] = R
    D[3:6, 3:6] = R
    for k in range(5):
        for l in range(5):
            D[6 + k, 6 + l] = np.sum(Y[k] * (R @ Y[l] @ R.T))
    return D


def test_rotation_covariance():
    rng = np.random.default_rng(11)
    pos, rad = _system(2, n=9, L=9.0)
    pos = pos - pos.mean(0) + 50.0          # a cluster far from any image
    L = 100.0
    A = rng.standard_normal((3, 3))
    R, _ = np.linalg.qr(A)
    if np.linalg.det(R) < 0:
        R[:, 0] *= -1
    D = _rep(R)
    theta = mpnn.init_params(4, head_scale=0.5)
    B = _iso_blocks(rad)
    b = rng.standard_normal((1, len(rad), 12))
    b[..., 11] = 0
    _, _, x0 = mpnn.loss_grad(theta, pos, rad, L, B, b, b, bf=False)
    pos_r = (pos - 50.0) @ R.T + 50.0
    b_r = b.copy()
    b_r[0, :, :11] = b[0, :, :11] @ D.T
    _, _, x0_r = mpnn.loss_grad(theta, pos_r, rad, L, B, b_r, b_r, bf=False)
    np.testing.assert_allclose(x0_r[0, :, :11], x0[0, :, :11] @ D.T, rtol=0, atol=1e-11 * np.abs(x0).max())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_structures_span_the_pair_mobility(seed):
    """Any 11x11 block that is a function of one displacement alone, such as
    the free-space pair coupling of the oracle, lies in the span of the 15
    structures of u = -d/|d|."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(3) * 2 + 1
    ai, aj = 1.0 + rng.random(), 1.0 + 2 * rng.random()
    Mb = ewald.pair_block_real(d, ai, aj, 0.0)[:11, :11]
    T = mpnn.structures(-d / np.linalg.norm(d)).reshape(15, -1)
    c, *_ = np.linalg.lstsq(T.T, Mb.reshape(-1), rcond=None)
    assert np.linalg.norm(c @ T - Mb.reshape(-1)) < 1e-12 * np.linalg.norm(Mb)
    # and the 15 are independent
    assert np.linalg.matrix_rank(T) == 15


def test_permutation_invariance():
    rng = np.random.default_rng(3)
    pos, rad = _system(4)
    theta = mpnn.init_params(9, head_scale=0.5)
    B = _aniso_blocks(rad, 2)
    b = rng.standard_normal((2, len(rad), 12))
    xs = rng.standard_normal((2, len(rad), 12))
    l1, g1, x1 = mpnn.loss_grad(theta, pos, rad, 8.0, B, b, xs, bf=False)
    pr = rng.permutation(len(rad))
    l2, g2, x2 = mpnn.loss_grad(theta, pos[pr], rad[pr], 8.0, B[pr], b[:, pr], xs[:, pr], bf=False)
    assert abs(l1 - l2) < 1e-12 * l1
    np.testing.assert_allclose(g2, g1, rtol=1e-9, atol=1e-12 * np.abs(g1).max())
    np.testing.assert_allclose(x2, x1[:, pr], rtol=1e-12, atol=1e-14)


def test_zero_heads_give_block_diagonal_guess():
    pos, rad = _system(5)
    p = mpnn.unpack(mpnn.init_params(1))
    for k in ("W_o", "b_o", "W_c", "b_c"):
        p[k][...] = 0.0
    B = _aniso_blocks(rad, 3)
    b = np.random.default_rng(0).standard_normal((1, len(rad), 12))
    _, _, x0 = mpnn.loss_grad(mpnn.pack(p), pos, rad, 8.0, B, b, b, bf=True)
    np.testing.assert_allclose(x0[0, :, :11], np.einsum("nab,nb->na", B[:, :11, :11], b[0, :, :11]), rtol=1e-12)


def test_graph_cutoff_and_features():
    pos = np.array([[1.0, 1.0, 1.0], [4.9, 1.0, 1.0], [1.0, 6.5, 1.0]])
    rad = np.array([1.0, 1.0, 2.0])
    g = mpnn.graph(pos, rad, 20.0)
    pairs = set(zip(g["src"].tolist(), g["dst"].tolist()))
    # 0-1: r = 3.9 < 4; 0-2: r = 5.5 < 6; 1-2: r = sqrt(3.9^2+5.5^2) = 6.74 > 6
    assert pairs == {(0, 1), (1, 0), (0, 2), (2, 0)}
    fn, fe = mpnn.features(g, rad)
    e = list(zip(g["src"], g["dst"])).index((0, 2))
    np.testing.assert_allclose(fe[e, :5], [5.5 / 3, 3 / 5.5, (3 / 5.5) ** 3, np.log(2.0), 2 / 3])
    np.testing.assert_allclose(fn[0, :4], [2 / 16, ((2 / 3.9) ** 3 + (3 / 5.5) ** 3) / 16,
                                           np.log1p(1 + 8) / 4, np.log(2.0) / 2])
