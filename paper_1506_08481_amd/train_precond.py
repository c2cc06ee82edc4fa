"""Training and evaluation driver of the learned far-field preconditioner.

Every numerical step runs in the HIP library (network forward and backward,
the method's own mobility products for the residual loss, Adam); this module
only generates the synthetic far-field problems and loops over them.

Training problems: bidisperse suspensions (radii 1 and lambda, lambda
uniform in [1, 4], large-sphere volume share uniform in [0.3, 0.7]) with N
log-uniform in [2000, 12000] and phi uniform in [0.1, 0.45], placed at random
without overlap; right-hand sides b i.i.d. N(0, 1) on the incompressible
components. Each training step takes one configuration with `nrhs`
right-hand sides; the loss is the mean relative residual
||b' - A x0||^2 / ||b'||^2 of the network's initial guess, with A applied by
the library's product in the configuration the autotuner picks for that
suspension (FP32, 1e-6 target).

Command line: python -m paper_1506_08481_amd.train_precond --out weights.bin
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import sys
import time

import numpy as np

from . import workloads as wl

NMIN, NMAX = 2000, 12000
PHI = (0.1, 0.45)
LAM = (1.0, 4.0)


def make_problem(k: int, seed: int):
    """Configuration k of the training set (deterministic in (k, seed))."""
    rng = np.random.default_rng([seed, k])
    for attempt in range(8):
        n = int(math.exp(rng.uniform(math.log(NMIN), math.log(NMAX))))
        phi = float(rng.uniform(*PHI))
        lam = float(rng.uniform(*LAM))
        y2 = float(rng.uniform(0.3, 0.7))
        s = wl.bidisperse(n, phi, seed * 100003 + 7 * k + attempt, a1=1.0, a2=lam, y2=y2)
        if s.L > 8.5 * s.radius.max():
            return s
    raise RuntimeError("no admissible configuration")


def _cfg_for(seasd, s, precision):
    return seasd.seasd_autotune(s.n, s.box, float(np.quantile(s.radius, 0.1)), float(s.radius.max()), 1e-6,
                                precision)


class ProblemPool:
    """Worker processes that place the training configurations. Create it
    before anything in the process touches the GPU (the workers are forked)."""

    def __init__(self, nconf: int, seed: int, procs: int = 16):
        self.nconf = nconf
        self.pool = mp.get_context("fork").Pool(procs)
        self.arrivals = self.pool.imap_unordered(_make_star, [(k, seed) for k in range(nconf)])

    def close(self):
        self.pool.close()
        self.pool.join()


def train(net, problems: ProblemPool, epochs: int = 12, nrhs: int = 8, lr: float = 5e-4, seed: int = 11,
          log=None):
    """Train `net` in place on the configurations `problems` delivers; returns
    the loss history (one entry per step)."""
    import torch

    from . import seasd
    dev = torch.device("cuda:0")
    eng = seasd.Seasd(0)
    history = []
    confs = []
    t0 = time.time()
    nconf = problems.nconf
    total_steps = nconf * epochs
    step = 0
    rng = np.random.default_rng(seed + 1)

    def one_step(c):
        nonlocal step
        s, P, R = c
        eng.set_config(**{f: getattr(_cfg_for(seasd, s, seasd.SEASD_FP32), f)
                          for f in ("grid", "P", "m", "xi", "rc_factor")},
                       precision=seasd.SEASD_FP32, checks=0)
        b = torch.randn((nrhs, s.n, 12), dtype=torch.float64, device=dev,
                        generator=None)
        b[..., 11] = 0.0
        frac = step / max(total_steps - 1, 1)
        lr_t = lr * (0.1 + 0.9 * 0.5 * (1.0 + math.cos(math.pi * frac)))   # cosine to lr/10
        loss = net.train_step(eng, P, R, s.box, b, lr=lr_t)
        history.append(loss)
        step += 1

    torch.manual_seed(seed)
    try:
        for s in problems.arrivals:   # first epoch as configurations arrive
            c = (s, torch.as_tensor(s.pos, device=dev), torch.as_tensor(s.radius, device=dev))
            confs.append(c)
            one_step(c)
            if log and len(confs) % 8 == 0:
                log(f"configs {len(confs)}/{nconf} steps {step} loss(last 8) {np.mean(history[-8:]):.4f} "
                    f"{time.time() - t0:.0f}s")
        for ep in range(1, epochs):
            for k in rng.permutation(len(confs)):
                one_step(confs[k])
            if log:
                log(f"epoch {ep + 1}/{epochs} steps {step} loss {np.mean(history[-len(confs):]):.4f} "
                    f"{time.time() - t0:.0f}s")
    finally:
        problems.close()
        eng.close()
    return history


def _make_star(args):
    return make_problem(*args)


def evaluate(net, s, tol: float = 1e-6, precision=None, seed: int = 5, repeats: int = 1):
    """Far-field solves of one suspension with the block-diagonal
    preconditioner and with the learned guess (same blocks); returns the stats
    of each (last repeat) and the solve wall time."""
    import torch

    from . import seasd
    if precision is None:
        precision = seasd.SEASD_FP32
    dev = torch.device("cuda:0")
    P = torch.as_tensor(s.pos, device=dev)
    R = torch.as_tensor(s.radius, device=dev)
    gen = np.random.default_rng(seed)
    b = gen.standard_normal((s.n, 12))
    b[:, 11] = 0.0
    B = torch.as_tensor(b, device=dev)
    cfg = _cfg_for(seasd, s, precision)
    out = {}
    xs = {}
    for name, pc in (("blockdiag", seasd.SEASD_PRECOND_BLOCKDIAG),
                     ("learned_guess", seasd.SEASD_PRECOND_LEARNED_GUESS)):
        eng = seasd.Seasd(0, **{f: getattr(cfg, f) for f in ("grid", "P", "m", "xi", "rc_factor")},
                          precision=precision, tol=tol, restart=50, max_iter=3000, precond=pc, checks=0)
        if pc != seasd.SEASD_PRECOND_BLOCKDIAG:
            eng.attach(net)
        eng.solve(P, R, s.box, B)   # warm-up: workspace, block fit
        torch.cuda.synchronize()
        for _ in range(repeats):
            t0 = time.perf_counter()
            x, st = eng.solve(P, R, s.box, B)
            torch.cuda.synchronize()
            st["wall_s"] = time.perf_counter() - t0
        xs[name] = x.cpu().numpy()
        out[name] = st
        eng.close()
    ref = xs["blockdiag"]
    for k in out:
        out[k]["rel_diff_vs_blockdiag"] = float(np.linalg.norm(xs[k] - ref) / np.linalg.norm(ref))
    out["config"] = {k: v for k, v in cfg.as_dict().items() if k in ("grid", "P", "m", "xi", "rc_factor")}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--configs", type=int, default=96)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--seed", type=int, default=11)
    args = ap.parse_args()
    problems = ProblemPool(args.configs, args.seed)   # before the GPU is touched
    from . import seasd
    net = seasd.Net(0, seed=args.seed)
    hist = train(net, problems, args.epochs, args.nrhs, args.lr, args.seed,
                 log=lambda m: print(m, file=sys.stderr, flush=True))
    net.save(args.out)
    print(json.dumps({"steps": len(hist), "loss_first": hist[0], "loss_last_epoch": float(np.mean(hist[-args.configs:]))}))


if __name__ == "__main__":
    main()
