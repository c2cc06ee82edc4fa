"""The learned preconditioner through the C ABI: network forward, initial
guess, residual loss and gradient against the FP64 reference network
(oracle/mpnn.py, with the same bfloat16 rounding of matrix-product operands,
and the oracle's converged Ewald sum as the operator), training on the GPU,
solves with the learned preconditioner, its fallback, and the weights file.

Tolerances (BF16 operands, FP32 accumulation on the GPU against FP64
accumulation in the reference): the two sides round the same operands, but
an FP32 sum that lands on the other side of a bfloat16 rounding boundary
changes that operand by 2^-8 relative; such flips are rare and their effect
averages out, so the initial guess agrees to 5e-4 relative, the loss to
1e-3 and every parameter tensor's gradient to 1e-2 relative (2-norm). The
same comparison without the rounding in the reference differs by about a
hundred times more, which shows the rounding is reproduced.
"""
import math
import os

import numpy as np
import pytest

from oracle import ewald, mpnn, solve
from paper_1506_08481_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_08481_amd import seasd
    return seasd


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _oracle_inverse_blocks(s):
    """Block-diagonal preconditioner blocks by the oracle: M_ii of each distinct
    radius alone in the cell, trace row and column replaced by the identity,
    inverted."""
    p = ewald.converged_params(s.box, s.radius, xi=0.6, tol_exp=6.0)
    out = np.zeros((s.n, 12, 12))
    for a in np.unique(s.radius):
        B = solve.self_image_block(a, s.box, p)
        B[11, :] = 0.0
        B[:, 11] = 0.0
        B[11, 11] = 1.0
        out[s.radius == a] = np.linalg.inv(B)
    return out


CFG = dict(grid=64, P=24, m=0.9 * math.sqrt(math.pi * 24), xi=0.6, rc_factor=5.0)


@pytest.fixture(scope="module")
def case():
    s = wl.bidisperse(150, 0.3, 515, a1=1.0, a2=1.5)
    rng = np.random.default_rng(516)
    b = rng.standard_normal((2, s.n, 12))
    b[..., 11] = 0.0
    B = _oracle_inverse_blocks(s)
    theta = mpnn.init_params(517, head_scale=0.3)
    p = mpnn.unpack(theta)
    for k in p:
        if k.startswith("b_"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    theta = mpnn.pack(p).astype(np.float32).astype(np.float64)
    return s, b, B, theta


def _oracle_A(s):
    """The 11x11 incompressible block of the oracle's converged Ewald sum."""
    p = ewald.converged_params(s.box, s.radius, xi=0.9, tol_exp=6.0)

    def Aop(v):
        x = np.zeros((s.n, 12))
        x[:, :11] = v[:, :11]
        return ewald.apply(s.pos, s.radius, s.box, x, p)[:, :11]
    return Aop


def test_forward_loss_gradient_match_reference(lib, case):
    s, b, B, theta = case
    assert s.L > 8 * s.radius.max()
    lo, go, x0o = mpnn.residual_loss_grad(theta, s.pos, s.radius, s.L, B, b, _oracle_A(s), bf=True)
    eng = lib.Seasd(0, **CFG)
    net = lib.Net(0, seed=1)
    net.set_params(theta.astype(np.float32))
    loss, grad, x0 = net.loss_grad(eng, _t(s.pos), _t(s.radius), s.box, _t(b), want_grad=True)
    x0 = x0.cpu().numpy()
    ex = np.linalg.norm(x0 - x0o) / np.linalg.norm(x0o)
    el = abs(loss - lo) / lo
    x0_exact = mpnn.x0_apply(*_exact_outputs(theta, s), mpnn.graph(s.pos, s.radius, s.L), B, b)
    ex_exact = np.linalg.norm(x0 - x0_exact) / np.linalg.norm(x0_exact)
    print(f"x0 rel {ex:.2e} (unrounded reference: {ex_exact:.2e}) loss {loss:.6e} vs {lo:.6e} rel {el:.2e}")
    off = 0
    errs = {}
    for name, shape in mpnn.layout():
        size = int(np.prod(shape))
        gg, gr = grad[off:off + size], go[off:off + size]
        off += size
        errs[name] = np.linalg.norm(gg - gr) / max(np.linalg.norm(gr), 1e-30)
        print(f"  grad {name:6s} |g| {np.linalg.norm(gr):.3e} rel {errs[name]:.2e}")
    assert ex < 5e-4 and el < 1e-3
    assert ex_exact > 10 * ex
    assert max(errs.values()) < 1e-2, errs
    net.close()
    eng.close()


def _exact_outputs(theta, s):
    g = mpnn.graph(s.pos, s.radius, s.L)
    fn, fe = mpnn.features(g, s.radius)
    act = mpnn.forward(theta, fn, fe, g, bf=False)
    return act["o"], act["c"]


def test_fresh_network_reproduces_block_diagonal_guess(lib, case):
    """Zero output layers: S = I and no pair terms, so x0 = B b exactly (the
    GPU's own blocks against the oracle's)."""
    s, b, B, theta = case
    p = mpnn.unpack(theta)
    for k in ("W_o", "b_o", "W_c", "b_c"):
        p[k][...] = 0.0
    eng = lib.Seasd(0, **CFG)
    net = lib.Net(0)
    net.set_params(mpnn.pack(p).astype(np.float32))
    _, _, x0 = net.loss_grad(eng, _t(s.pos), _t(s.radius), s.box, _t(b), want_loss=False)
    ref = np.einsum("nab,qnb->qna", B[:, :11, :11], b[:, :, :11])
    e = np.linalg.norm(x0.cpu().numpy()[..., :11] - ref) / np.linalg.norm(ref)
    print("block-diagonal guess rel", e)
    assert e < 1e-8
    net.close()
    eng.close()


def _solve(lib, s, b, precond, net=None, tol=1e-8):
    eng = lib.Seasd(0, tol=tol, restart=50, max_iter=600, precond=precond, compressible=1, **CFG)
    if net is not None:
        eng.attach(net)
    x, st = eng.solve(_t(s.pos), _t(s.radius), s.box, _t(b))
    out = x.cpu().numpy()
    eng.close()
    return out, st


def test_training_lowers_loss_and_learned_solve_converges(lib, case):
    s, b, _, _ = case
    rng = np.random.default_rng(518)
    train = rng.standard_normal((8, s.n, 12))
    train[..., 11] = 0.0
    eng = lib.Seasd(0, **CFG)
    net = lib.Net(0, seed=7)
    P, R, Bt = _t(s.pos), _t(s.radius), _t(train)
    losses = [net.train_step(eng, P, R, s.box, Bt, lr=2e-3) for _ in range(60)]
    held, _, _ = net.loss_grad(eng, P, R, s.box, _t(b))
    print("loss", losses[0], "->", losses[-1], "held-out", held)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.7 * losses[0] and held < 0.7 * losses[0]
    eng.close()
    x_bd, st_bd = _solve(lib, s, b[0], lib.SEASD_PRECOND_BLOCKDIAG)
    for mode in (lib.SEASD_PRECOND_LEARNED_GUESS,):
        x_l, st_l = _solve(lib, s, b[0], mode, net)
        print("block-diagonal", st_bd)
        print("learned mode", mode, st_l)
        assert st_l["converged"] == 1 and st_l["precond_used"] == mode
        assert st_l["guess_used"] == 1 and st_l["initial_residual"] < st_bd["initial_residual"]
        assert st_l["true_residual"] <= 1e-8
        assert np.linalg.norm(x_l - x_bd) / np.linalg.norm(x_bd) < 1e-6
    net.close()


def test_rejected_network_falls_back_to_block_diagonal(lib, case):
    s, b, _, _ = case
    bb = b[0].copy()
    bb[:, 11] = 0.0
    net = lib.Net(0)
    p = net.params()
    p[:] = np.nan
    net.set_params(p)
    x_bd, st_bd = _solve(lib, s, bb, lib.SEASD_PRECOND_BLOCKDIAG)
    x_l, st_l = _solve(lib, s, bb, lib.SEASD_PRECOND_LEARNED_GUESS, net)
    print(st_l)
    assert st_l["code"] == lib.SEASD_W_PRECOND_FALLBACK
    assert st_l["precond_used"] == lib.SEASD_PRECOND_BLOCKDIAG and st_l["guess_used"] == 0
    assert st_l["iterations"] == st_bd["iterations"]
    np.testing.assert_allclose(x_l, x_bd, rtol=0, atol=1e-12 * np.abs(x_bd).max())
    net.close()


def test_weights_file_roundtrip_and_checksum(lib, tmp_path):
    net = lib.Net(0, seed=3)
    p = net.params()
    f = str(tmp_path / "w.bin")
    net.save(f)
    other = lib.Net(0, seed=4)
    other.load(f)
    np.testing.assert_array_equal(other.params(), p)
    raw = bytearray(open(f, "rb").read())
    raw[100] ^= 0x40
    open(f + ".bad", "wb").write(bytes(raw))
    open(f + ".short", "wb").write(bytes(raw[:-9]))
    for bad in (f + ".bad", f + ".short", str(tmp_path / "missing.bin")):
        with pytest.raises(lib.SeasdError) as ei:
            other.load(bad)
        assert ei.value.code == lib.SEASD_E_FORMAT
    np.testing.assert_array_equal(other.params(), p)   # unchanged by the failed loads
    net.close()
    other.close()


WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1506_08481_amd",
                       "weights", "precond_mpnn.bin")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights in the tree")
def test_trained_weights_gain_on_unseen_suspension(lib):
    """The shipped network on a suspension it was not trained on (N = 6000,
    bidisperse 1:2, phi = 0.35, FP64 product): the learned guess starts GMRES
    well below the zero guess, both solves reach the tolerance on the true
    residual, and the learned guess takes fewer GMRES iterations than the
    block-diagonal method alone (the gain the network brings; a few per cent,
    see the design notes on why a per-sphere guess cannot reach further)."""
    from paper_1506_08481_amd import train_precond
    s = wl.bidisperse(6000, 0.35, 9191, a1=1.0, a2=2.0)
    eng = lib.Seasd(0)
    eng.precond_load(WEIGHTS)
    net = lib.Net(0)
    net.load(WEIGHTS)
    res = train_precond.evaluate(net, s, tol=1e-6, precision=lib.SEASD_FP64)
    for k in ("blockdiag", "learned_guess"):
        print(k, {q: res[k][q] for q in ("iterations", "matvecs", "initial_residual", "true_residual", "wall_s")})
    bd, lg = res["blockdiag"], res["learned_guess"]
    assert bd["converged"] == 1 and lg["converged"] == 1
    print("iterations saved by the learned guess:", bd["iterations"] - lg["iterations"])
    assert lg["guess_used"] == 1 and lg["initial_residual"] < 0.8
    assert lg["iterations"] < bd["iterations"]
    assert lg["rel_diff_vs_blockdiag"] < 1e-4
    net.close()
    eng.close()
