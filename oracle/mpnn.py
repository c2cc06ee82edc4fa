"""Reference of the learned far-field preconditioner network (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper has no learned component: its far-field preconditioner is the
block-diagonal approximation of Sec. 4.2 (each sphere with its own periodic
images, block inverted exactly). This module is the plain definition of the
project's message-passing network that sits on top of those inverse blocks
B_i and predicts
  (i)  per-sphere corrections: group scalings s_i (force, torque, stresslet)
       that turn B_i into S_i B_i S_i, and
  (ii) an initial guess x0 = S B S b + sum over neighbour pairs of
       sigma_i * Q(c_ij, u_ij) (sigma_j * b_j) for GMRES,
written as formulas over explicit arrays with numpy matrix products as the
only library steps. Every matrix product rounds both operands to bfloat16
when bf=True (the library's GEMMs take BF16 operands and accumulate in FP32);
with bf=False everything is FP64 and the gradient is checked by finite
differences.

Definitions (edges i -> j, i != j, minimum image, |r_ij| < 2 (a_i + a_j)):
  u_ij   = (x_j - x_i) / |x_j - x_i|
  e_ij   = [rho, 1/rho, 1/rho^3, log(a_j/a_i), a_j/(a_i+a_j), 0 ...] (16),
           rho = |r_ij| / (a_i + a_j)
  x_i    = [deg/16, sum_j rho^-3/16, log1p(sum_j (a_j/a_i)^3)/4,
            mean_j log(a_j/a_i), 0 ...] (16)
  h      = relu(x W_in + b_in)
  two layers:  [U|V] = h W_uv;  a_ij = relu(U_i + V_j + e_ij W_e + b_a);
               m_ij = relu(a_ij W_m + b_m);  g_i = sum_j m_ij / 16;
               h   <- h + relu([h|g] W_h + b_h)
  o_i    = h W_o + b_o   (o_i[0:3]: log-scalings of the F, T, S groups)
  c_ij   = m_ij W_c + b_c (c_ij[0:15]: coefficients of the 15 structures)
  sigma_i[c] = sqrt(B_i[c, c]),  s_i[c] = exp(o_i[group(c)] / 2)  (c < 11)
  x0_i   = s_i * B_i (s_i * b_i) + sum_j sigma_i * (sum_k c_ijk T_k(u_ij)) (sigma_j * b_j)
  loss   = mean over right-hand sides of ||b' - A x0||^2 / ||b'||^2 (the
           relative residual of the guess, A the 11x11 incompressible block
           of the mobility); an error loss against solutions x*,
           mean ((x0 - x*) / sigma^2)^2, is also provided
The T_k are the 15 rotation-covariant 11x11 maps between (F, T, S) and
(U, Omega, E) that a direction u allows (structures()).
"""
from __future__ import annotations

import numpy as np

from .symbols import traceless_basis

H = 64
FN = 16
FE = 16
NO = 16
EDGE_CUT = 2.0
AGG = 1.0 / 16.0


def layout():
    """(name, shape) of every parameter in the flat vector, in order. Weights
    are stored row-major as [fan_in, fan_out] (y = x W)."""
    out = [("W_in", (FN, H)), ("b_in", (H,))]
    for l in range(2):
        out += [(f"W_uv{l}", (H, 2 * H)), (f"W_e{l}", (FE, H)), (f"b_a{l}", (H,)),
                (f"W_m{l}", (H, H)), (f"b_m{l}", (H,)), (f"W_h{l}", (2 * H, H)), (f"b_h{l}", (H,))]
    out += [("W_o", (H, NO)), ("b_o", (NO,)), ("W_c", (H, NO)), ("b_c", (NO,))]
    return out


def param_count() -> int:
    return int(sum(np.prod(s) for _, s in layout()))


def unpack(theta):
    p, off = {}, 0
    for name, shape in layout():
        size = int(np.prod(shape))
        p[name] = np.asarray(theta[off:off + size], dtype=np.float64).reshape(shape)
        off += size
    return p


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in layout()])


def bf16(x):
    """Round to bfloat16 the way the library does: to float32 first (nearest
    even), then to 8 mantissa bits (nearest even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(x, w, bf):
    return (bf16(x) @ bf16(w)) if bf else (x @ w)


# ---------------------------------------------------------------------------
# graph and features

def graph(pos, rad, L):
    """All directed edges by brute force, ordered by (i, j)."""
    n = pos.shape[0]
    d = pos[None, :, :] - pos[:, None, :]            # x_j - x_i
    d -= L * np.round(d / L)
    r = np.linalg.norm(d, axis=2)
    ai, aj = rad[:, None], rad[None, :]
    mask = (r < EDGE_CUT * (ai + aj)) & ~np.eye(n, dtype=bool)
    src, dst = np.nonzero(mask)
    rr = r[src, dst]
    return {"n": n, "src": src, "dst": dst, "r": rr, "u": d[src, dst] / rr[:, None]}


def features(g, rad):
    src, dst, r = g["src"], g["dst"], g["r"]
    ai, aj = rad[src], rad[dst]
    rho = r / (ai + aj)
    fe = np.zeros((len(src), FE))
    fe[:, 0] = rho
    fe[:, 1] = 1.0 / rho
    fe[:, 2] = rho ** -3
    fe[:, 3] = np.log(aj / ai)
    fe[:, 4] = aj / (ai + aj)
    n = g["n"]
    deg = np.bincount(src, minlength=n).astype(np.float64)
    fn = np.zeros((n, FN))
    fn[:, 0] = deg / 16.0
    fn[:, 1] = np.bincount(src, weights=rho ** -3, minlength=n) / 16.0
    fn[:, 2] = np.log1p(np.bincount(src, weights=(aj / ai) ** 3, minlength=n)) / 4.0
    sl = np.bincount(src, weights=np.log(aj / ai), minlength=n)
    fn[:, 3] = np.where(deg > 0, sl / np.maximum(deg, 1.0), 0.0)
    return fn, fe


# ---------------------------------------------------------------------------
# the 15 covariant structures

def structures(u) -> np.ndarray:
    """T[k] (11x11) for unit vector u; rows (U, Omega, E), columns (F, T, S),
    E and S in the orthonormal traceless coordinates."""
    Y = traceless_basis()
    T = np.zeros((15, 11, 11))
    uu = np.outer(u, u)
    X = np.array([[0.0, -u[2], u[1]], [u[2], 0.0, -u[0]], [-u[1], u[0], 0.0]])   # X v = u x v
    Yu = np.einsum("kab,b->ka", Y, u)           # row k: Y_k u
    q = np.einsum("a,kab,b->k", u, Y, u)       # u . Y_k u
    F, Tq, S = slice(0, 3), slice(3, 6), slice(6, 11)
    T[0][F, F] = np.eye(3)
    T[1][F, F] = uu
    T[2][F, Tq] = X
    T[3][Tq, F] = X
    T[4][Tq, Tq] = np.eye(3)
    T[5][Tq, Tq] = uu
    T[6][F, S] = Yu.T
    T[7][F, S] = np.outer(u, q)
    T[8][S, F] = Yu
    T[9][S, F] = np.outer(q, u)
    T[10][Tq, S] = X @ Yu.T
    T[11][S, Tq] = (X @ Yu.T).T
    T[12][S, S] = np.eye(5)
    T[13][S, S] = Yu @ Yu.T
    T[14][S, S] = np.outer(q, q)
    return T


GROUP = np.array([0, 0, 0, 1, 1, 1, 2, 2, 2, 2, 2])


# ---------------------------------------------------------------------------
# network

def forward(theta, fn, fe, g, bf=True):
    p = unpack(theta)
    src, dst, n = g["src"], g["dst"], g["n"]
    act = {}
    z0 = _mm(fn, p["W_in"], bf) + p["b_in"]
    h = np.maximum(z0, 0.0)
    act["h0"] = h
    for l in range(2):
        uv = _mm(h, p[f"W_uv{l}"], bf)
        a = np.maximum(uv[src, :H] + uv[dst, H:] + _mm(fe, p[f"W_e{l}"], bf) + p[f"b_a{l}"], 0.0)
        m = np.maximum(_mm(a, p[f"W_m{l}"], bf) + p[f"b_m{l}"], 0.0)
        gg = np.zeros((n, H))
        np.add.at(gg, src, m)
        gg *= AGG
        hg = np.concatenate([h, gg], axis=1)
        r = np.maximum(_mm(hg, p[f"W_h{l}"], bf) + p[f"b_h{l}"], 0.0)
        act[f"hin{l}"], act[f"a{l}"], act[f"m{l}"], act[f"g{l}"], act[f"r{l}"] = h, a, m, gg, r
        h = h + r
    act["h2"] = h
    act["o"] = _mm(h, p["W_o"], bf) + p["b_o"]
    act["c"] = _mm(act["m1"], p["W_c"], bf) + p["b_c"]
    return act


def _pieces(o, c, g, Binv):
    B = Binv[:, :11, :11]
    sig = np.sqrt(np.einsum("ncc->nc", B))
    s = np.exp(0.5 * o[:, GROUP])                          # [n, 11]
    Tk = np.stack([structures(u) for u in g["u"]]) if len(g["src"]) else np.zeros((0, 15, 11, 11))
    return B, sig, s, Tk


def x0_apply(o, c, g, Binv, b):
    """x0 for every right-hand side; Binv: [n, 12, 12]; b: [nrhs, n, 12]."""
    src, dst = g["src"], g["dst"]
    B, sig, s, Tk = _pieces(o, c, g, Binv)
    Q = np.einsum("ek,ekab->eab", c[:, :15], Tk)           # [E, 11, 11]
    x0 = np.zeros(b.shape[:2] + (12,))
    for q in range(b.shape[0]):
        bq = b[q, :, :11]
        y = s * np.einsum("nab,nb->na", B, s * bq)
        y_e = sig[src] * np.einsum("eab,eb->ea", Q, sig[dst] * bq[dst])
        np.add.at(y, src, y_e)
        x0[q, :, :11] = y
    return x0


def x0_vjp(o, c, g, Binv, b, gx):
    """Gradients with respect to o and c of sum(gx * x0)."""
    src, dst = g["src"], g["dst"]
    B, sig, s, Tk = _pieces(o, c, g, Binv)
    do, dc = np.zeros_like(o), np.zeros_like(c)
    for q in range(b.shape[0]):
        bq, gq = b[q, :, :11], gx[q, :, :11]
        Bsb = np.einsum("nab,nb->na", B, s * bq)
        dLds = gq * Bsb + bq * np.einsum("nba,nb->na", B, s * gq)
        np.add.at(do.T, GROUP, (0.5 * s * dLds).T)
        dc[:, :15] += np.einsum("ea,ekab,eb->ek", sig[src] * gq[src], Tk, sig[dst] * bq[dst])
    return do, dc


def x0_and_loss(o, c, g, Binv, b, xstar=None):
    """x0 and, with x*, the error loss mean(((x0 - x*) / sigma^2)^2) and its
    gradient with respect to o and c."""
    x0 = x0_apply(o, c, g, Binv, b)
    if xstar is None:
        return x0, 0.0, np.zeros_like(o), np.zeros_like(c)
    sig2 = np.einsum("ncc->nc", Binv[:, :11, :11])
    cnt = b.shape[0] * g["n"] * 11
    eps = (x0[..., :11] - xstar[..., :11]) / sig2
    gx = np.zeros_like(x0)
    gx[..., :11] = 2.0 * eps / sig2 / cnt
    do, dc = x0_vjp(o, c, g, Binv, b, gx)
    return x0, float((eps ** 2).sum()) / cnt, do, dc


def residual_loss(x0, b, Aop):
    """mean over right-hand sides of ||b' - A x0||^2 / ||b'||^2 (b' = b on the
    11 incompressible components) and its gradient with respect to x0 (A
    symmetric). Aop maps [n, 12] (trace ignored) to [n, 11]."""
    nrhs = b.shape[0]
    loss, gx = 0.0, np.zeros_like(x0)
    for q in range(nrhs):
        bq = b[q, :, :11]
        nb2 = float((bq ** 2).sum())
        r = bq - Aop(x0[q])
        loss += float((r ** 2).sum()) / nb2 / nrhs
        rr = np.zeros_like(x0[q])
        rr[:, :11] = r
        gx[q, :, :11] = -2.0 * Aop(rr) / nb2 / nrhs
    return loss, gx


def backward(theta, fn, fe, g, act, do, dc, bf=True):
    p = unpack(theta)
    src, dst, n = g["src"], g["dst"], g["n"]
    gr = {k: np.zeros_like(v) for k, v in p.items()}

    def lin_back(x, w, dz):
        """y = x w (+ b): returns dx, dw, db."""
        dx = (bf16(dz) @ bf16(w).T) if bf else dz @ w.T
        dw = (bf16(x).T @ bf16(dz)) if bf else x.T @ dz
        return dx, dw, dz.sum(axis=0)

    dm_c, gr["W_c"], gr["b_c"] = lin_back(act["m1"], p["W_c"], dc)
    dh, gr["W_o"], gr["b_o"] = lin_back(act["h2"], p["W_o"], do)
    dm_extra = dm_c
    for l in (1, 0):
        hin, a, m, gg, r = act[f"hin{l}"], act[f"a{l}"], act[f"m{l}"], act[f"g{l}"], act[f"r{l}"]
        dz_h = dh * (r > 0)
        dhg, gr[f"W_h{l}"], gr[f"b_h{l}"] = lin_back(np.concatenate([hin, gg], axis=1), p[f"W_h{l}"], dz_h)
        dh_in = dh + dhg[:, :H]
        dm = dhg[src, H:] * AGG + dm_extra
        dz_m = dm * (m > 0)
        da, gr[f"W_m{l}"], gr[f"b_m{l}"] = lin_back(a, p[f"W_m{l}"], dz_m)
        dz_a = da * (a > 0)
        _, gr[f"W_e{l}"], gr[f"b_a{l}"] = lin_back(fe, p[f"W_e{l}"], dz_a)
        duv = np.zeros((n, 2 * H))
        np.add.at(duv[:, :H], src, dz_a)
        np.add.at(duv[:, H:], dst, dz_a)
        dx, gr[f"W_uv{l}"], _ = lin_back(hin, p[f"W_uv{l}"], duv)
        dh = dh_in + dx
        dm_extra = 0.0
    dz0 = dh * (act["h0"] > 0)
    _, gr["W_in"], gr["b_in"] = lin_back(fn, p["W_in"], dz0)
    return pack(gr)


def loss_grad(theta, pos, rad, L, Binv, b, xstar, bf=True):
    """Error loss, flat gradient and x0 for one configuration and nrhs pairs
    (b, x*)."""
    g = graph(pos, rad, L)
    fn, fe = features(g, rad)
    act = forward(theta, fn, fe, g, bf)
    x0, loss, do, dc = x0_and_loss(act["o"], act["c"], g, Binv, b, xstar)
    grad = backward(theta, fn, fe, g, act, do, dc, bf)
    return loss, grad, x0


def residual_loss_grad(theta, pos, rad, L, Binv, b, Aop, bf=True):
    """The training loss: relative residual of the guess, mean over right-hand
    sides of ||b' - A x0||^2 / ||b'||^2, its flat gradient and x0."""
    g = graph(pos, rad, L)
    fn, fe = features(g, rad)
    act = forward(theta, fn, fe, g, bf)
    x0 = x0_apply(act["o"], act["c"], g, Binv, b)
    loss, gx = residual_loss(x0, b, Aop)
    do, dc = x0_vjp(act["o"], act["c"], g, Binv, b, gx)
    grad = backward(theta, fn, fe, g, act, do, dc, bf)
    return loss, grad, x0


def init_params(seed: int, head_scale: float = 0.01) -> np.ndarray:
    """Uniform(-sqrt(6/fan_in), +) weights (fan_in counts only the used
    inputs), zero biases, output heads scaled by head_scale."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {}
    used = {"W_in": 4, "W_e0": 5, "W_e1": 5}
    for name, shape in layout():
        if name.startswith("b_"):
            p[name] = np.zeros(shape)
            continue
        fan = used.get(name, shape[0])
        lim = np.sqrt(6.0 / fan)
        w = rng.uniform(-lim, lim, size=shape)
        if name in ("W_in",):
            w[4:] = 0.0
        if name.startswith("W_e"):
            w[5:] = 0.0
        if name in ("W_o", "W_c"):
            w *= head_scale
        p[name] = w
    return pack(p)
