#!/usr/bin/env python3
"""Throughput of the Spectral Ewald grand-mobility product on one MI355X.

Workload: N = 100,000 monodisperse spheres (a = 1) at volume fraction 0.4 in a
periodic cube (L = 101.55), random non-overlapping placement; moments x drawn
i.i.d. N(0, 1); grid 256^3; spreading, FFTs and gather in FP32, pair sum in
FP64. One step = one full product y = M x (binning, real-space pair sum,
spreading, five FFT passes with the k-space multiply, gather), inputs resident
in HBM. Parameters (xi, r_c, P, m) are chosen among a few candidates as the
fastest one whose relative error against the FP64 GPU product is below 1e-6.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3     # published: counts packed two-wide FP32 FMAs
PEAK_FP64_TFLOPS = 78.6
# The library is compiled with packed FP32 instructions disabled, so its FP32
# vector code issues one FMA per lane and clock: 256 CUs x 4 SIMDs x 16 lanes
# x 2 flops x 2.4 GHz = 78.6 TFLOP/s, the ALU ceiling its FP32 kernels can reach.
PEAK_FP32_SCALAR_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# (xi, rc_factor, P, m / sqrt(pi P))
CANDIDATES = [
    (0.8, 3.0, 16, 0.85),
    (0.7, 3.5, 16, 0.95),
    (0.85, 2.82, 16, 0.85),
]
REF = (0.7, 3.5, 18, 0.95)   # FP64 reference product (SE error ~1e-8)


# HBM bytes per launch measured with the byte counters (FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0; the factors come from a 2 GiB elementwise kernel of known
# traffic profiled in the same runs), for the kernel versions and the
# configuration (phase, grid, P) recorded in
# profiles/product_n100000_phi0.4_grid256_traffic.md. Any other configuration
# reports null.
MEASURED_TRAFFIC = {
    ("spread", 256, 16): 322.4e6,
    ("gather", 256, 16): 995.4e6,
}


def phase_cost(phase, n, M, P, s_bytes, pairs):
    """Algorithmic bytes and flops of one launch of a phase: FFT passes read
    and write the 4-field grid once, 8 M^3 s bytes; spreading writes the grid
    once (4 M^3 s) and reads the binned particles (16 doubles each); gather
    reads the grid once (4 M^3 s) and the particles (28 doubles); flops
    counted from the kernels' arithmetic per sphere: spreading 71 per window
    column (its 13 z-polynomial coefficients) plus 26 per window point (13
    multiply-adds into the four fields), gather about 130 per window column
    (moment polynomials and 13 compensated sums) plus 26 per window point (13
    multiply-adds of the z moments); the pair sum costs about 700 FP64 flops
    per pair within r_c."""
    g = M ** 3
    if phase.startswith("fft"):
        return {"bytes": 8 * g * s_bytes, "flops": 0.0}
    if phase == "spread":
        return {"bytes": 4 * g * s_bytes + n * 16 * 8, "flops": n * (71.0 * P ** 2 + 26.0 * P ** 3)}
    if phase == "gather":
        return {"bytes": 4 * g * s_bytes + n * 28 * 8, "flops": n * (130.0 * P ** 2 + 26.0 * P ** 3)}
    if phase == "pair":
        return {"bytes": n * 28 * 8, "flops": 700.0 * pairs}
    return {"bytes": n * 64, "flops": 0.0}


def count_pairs(pos, rad, L, rc_factor):
    from scipy.spatial import cKDTree
    tree = cKDTree(np.mod(pos, L), boxsize=L)
    rmax = rc_factor * 2.0 * float(rad.max())
    pr = tree.query_pairs(rmax, output_type="ndarray")
    d = pos[pr[:, 0]] - pos[pr[:, 1]]
    d -= L * np.round(d / L)
    r = np.linalg.norm(d, axis=1)
    keep = r < rc_factor * (rad[pr[:, 0]] + rad[pr[:, 1]])
    return 2 * int(np.count_nonzero(keep))   # ordered pairs


def host_cores():
    """Cores this process may use (the CPU share of the host), at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_init(inputs):
    global _ORACLE_INPUTS
    _ORACLE_INPUTS = inputs


def _oracle_warm(_):
    from oracle import ewald  # noqa: F401  (imports paid before the timed runs)
    return 0


def _oracle_targets(args):
    """One worker of the sampled oracle product: all spheres of the benchmark
    workload are sources, the sum is evaluated at the given targets."""
    targets, xi, tol_exp = args
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)
    from oracle import ewald
    s, x = _ORACLE_INPUTS
    p = ewald.converged_params(s.box, s.radius, xi=xi, tol_exp=tol_exp)
    t0 = time.perf_counter()
    ewald.apply(s.pos, s.radius, s.box, x, p, targets=targets)
    return time.perf_counter() - t0


_ORACLE_INPUTS = None
ORACLE_XI, ORACLE_TOL_EXP = 0.1, 3.7
ORACLE_TARGETS_PER_WORKER = (1, 9)


def cpu_baseline(s_large=None, x_large=None):
    """The FP64 oracle (numpy classical Ewald sum, the test reference) timed on
    the host cores.

    * small workload in full: N = 100, phi = 0.1, one converged product
      (both Gaussian tails at exp(-42)), median of 3, BLAS on all cores;
    * the benchmark workload sampled: all N = 1e5 spheres are sources, the
      oracle evaluates the sum at a few targets in `cores` worker processes
      (one BLAS thread each, targets split between them), with both tails at
      exp(-3.7^2) = 1.1e-6, the accuracy the metric asks for. Two runs, one
      and nine targets per worker, separate the cost every worker pays once
      (structure sums over all sources, t_fixed) from the cost per target
      (t_target); the full product on the same cores is t_fixed +
      ceil(N / cores) t_target. That extrapolation in targets is the only
      scaling; `value` is its inverse."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle import ewald
    from paper_1506_08481_amd import workloads as wl
    cores = host_cores()
    small = wl.config_small()
    xs = wl.force_moments(small.n, 1000)
    ts = []
    with threadpool_limits(limits=cores):
        p = ewald.converged_params(small.box, small.radius, xi=0.5, tol_exp=6.5)
        for _ in range(3):
            t0 = time.perf_counter()
            ewald.apply(small.pos, small.radius, small.box, xs, p)
            ts.append(time.perf_counter() - t0)
    t_small = float(np.median(ts))

    if s_large is None:
        s_large = wl.config_large(seed=3000)
        x_large = wl.force_moments(s_large.n, 3001)
    n = s_large.n
    rng = np.random.default_rng(5)
    walls = []
    # fresh interpreters (spawn): the workers never touch the GPU
    with mp.get_context("spawn").Pool(cores, initializer=_oracle_init, initargs=((s_large, x_large),)) as pool:
        pool.map(_oracle_warm, range(cores))
        for per in ORACLE_TARGETS_PER_WORKER:
            tg = rng.choice(n, cores * per, replace=False)
            jobs = [(tg[w * per:(w + 1) * per], ORACLE_XI, ORACLE_TOL_EXP) for w in range(cores)]
            t0 = time.perf_counter()
            pool.map(_oracle_targets, jobs)
            walls.append(time.perf_counter() - t0)
    d_per = ORACLE_TARGETS_PER_WORKER[1] - ORACLE_TARGETS_PER_WORKER[0]
    t_target = max(walls[1] - walls[0], 1e-9) / d_per
    t_fixed = max(walls[0] - ORACLE_TARGETS_PER_WORKER[0] * t_target, 0.0)
    t_full = t_fixed + math.ceil(n / cores) * t_target
    return {"value": 1.0 / t_full, "unit": "matvecs/s", "cores": cores, "kind": "oracle",
            "cpu_model": host_cpu_model(),
            "sample": (f"FP64 numpy oracle (classical Ewald sum) on {cores} host cores ({host_cpu_model()}). "
                       f"Benchmark workload N={n}: all spheres as sources, the sum at "
                       f"{ORACLE_TARGETS_PER_WORKER[0] * cores} and {ORACLE_TARGETS_PER_WORKER[1] * cores} "
                       f"targets ({cores} worker processes, xi={ORACLE_XI}, tails exp(-{ORACLE_TOL_EXP}^2)) took "
                       f"{walls[0]:.1f} s and {walls[1]:.1f} s: fixed {t_fixed:.1f} s + {t_target:.2f} s per "
                       f"target per worker, so a full product is {t_full:.0f} s on these cores "
                       f"(extrapolated in targets). Small workload N=100 in full (converged): "
                       f"{t_small:.3f} s per product."),
            "small_workload_s_per_product": t_small,
            "large_sample_walls_s": walls, "large_full_product_s_estimate": t_full}


def _place_batch(k, seed):
    from paper_1506_08481_amd import workloads as wl
    return wl.batch_member(k, seed)


def bench_batch(args):
    """256 independent suspensions, N log-uniform in [500, 8000], radii
    lognormal (median 1, sigma 0.2), phi uniform in [0.1, 0.45], each with its
    own cell and grid; all products in one hipGraph launch, FP32, autotuned."""
    import multiprocessing as mp

    import torch

    from paper_1506_08481_amd import seasd
    from paper_1506_08481_amd import workloads as wl
    nsys = 256
    t0 = time.time()
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        sus = pool.starmap(_place_batch, [(k, 4000) for k in range(nsys)])
    offs = np.concatenate([[0], np.cumsum([s.n for s in sus])])
    pos = np.concatenate([s.pos for s in sus])
    rad = np.concatenate([s.radius for s in sus])
    x = wl.force_moments(int(offs[-1]), 4001)
    print(f"setup: {nsys} suspensions, {offs[-1]} spheres, placement {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    eng = seasd.Seasd(0, precision=seasd.SEASD_FP32, checks=0)
    t0 = time.time()
    plan = seasd.Batch(eng, offs, torch.as_tensor(pos, device=dev), torch.as_tensor(rad, device=dev),
                       [s.box for s in sus], target=1e-6)
    t_plan = time.time() - t0
    X = torch.as_tensor(x, device=dev)
    Y = torch.empty_like(X)
    for _ in range(args.warmup):
        plan.apply(X, Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(X, Y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    cfgs = plan.configs()
    grids = {}
    for c in cfgs:
        grids[c.grid[0]] = grids.get(c.grid[0], 0) + 1
    out = {"metric": "batched sphere-products/s (256 suspensions, one graph launch)",
           "value": float(offs[-1]) / dt, "unit": "sphere-products/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "256 suspensions, N log-uniform [500, 8000], radii lognormal(1, 0.2), "
                                  "phi U[0.1, 0.45], autotuned FP32", "spheres": int(offs[-1]),
                      "grids": {str(k): v for k, v in sorted(grids.items())}},
           "plan_build_s": t_plan}
    plan.close()
    eng.close()
    print(json.dumps(out))


def bench_solve(args):
    """N = 10,000 bidisperse spheres (radii 1 and 2, equal volume fraction per
    species, phi = 0.3), grid 128^3, FP64, right-hand side N(0, 1): far-field
    GMRES solve to relative residual 1e-8 with and without the block-diagonal
    preconditioner, and with FP32 products inside the Arnoldi cycles (FP64
    restart residuals, precision SEASD_MIXED)."""
    import torch

    from paper_1506_08481_amd import seasd
    from paper_1506_08481_amd import workloads as wl
    s = wl.config_bidisperse_solve()
    b = wl.force_moments(s.n, 2001)
    dev = torch.device("cuda:0")
    P_, R_, B_ = (torch.as_tensor(a, device=dev) for a in (s.pos, s.radius, b))
    c = seasd.seasd_autotune(s.n, s.box, 1.0, 2.0, 1e-8, seasd.SEASD_FP64)
    res, xs = {}, {}
    for name, pc, prec in (("blockdiag", seasd.SEASD_PRECOND_BLOCKDIAG, seasd.SEASD_FP64),
                           ("none", seasd.SEASD_PRECOND_NONE, seasd.SEASD_FP64),
                           ("mixed_blockdiag", seasd.SEASD_PRECOND_BLOCKDIAG, seasd.SEASD_MIXED)):
        eng = seasd.Seasd(0, grid=128, P=c.P, m=c.m, xi=c.xi, rc_factor=c.rc_factor, precision=prec,
                          tol=1e-8, restart=50, max_iter=1500, precond=pc, checks=1)
        eng.solve(P_, R_, s.box, B_)   # warm-up (allocation, code load)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = eng.solve(P_, R_, s.box, B_)
        torch.cuda.synchronize()
        st["wall_s"] = time.perf_counter() - t0
        res[name] = st
        xs[name] = x
        eng.close()
    res["mixed_blockdiag"]["rel_diff_vs_fp64_solution"] = float(
        torch.linalg.norm(xs["mixed_blockdiag"] - xs["blockdiag"]) / torch.linalg.norm(xs["blockdiag"]))
    out = {"metric": "far-field solve time, N=1e4 bidisperse phi=0.3, tol 1e-8",
           "value": res["blockdiag"]["wall_s"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": res["blockdiag"]["wall_s"] * 1e3, "higher_is_better": False, "scaling": "strong",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "bidisperse N=10000 (radii 1, 2) phi=0.3 grid 128^3 FP64 GMRES(50) tol 1e-8",
                      "xi": c.xi, "rc_factor": c.rc_factor, "P": c.P, "m": c.m},
           "solves": res}
    print(json.dumps(out))


def bench_learned(args):
    """Train the learned preconditioner on the GPU (synthetic bidisperse far-field
    problems, see paper_1506_08481_amd/train_precond.py), then solve one unseen
    suspension, N = 50,000 bidisperse (radii 1 and 2, equal volume per
    species), phi = 0.35, to relative residual 1e-6 with the block-diagonal
    preconditioner and with the learned one; reports iterations and wall time,
    also with FP32 products in the Arnoldi steps (precision SEASD_MIXED)."""
    from paper_1506_08481_amd import train_precond as tp
    from paper_1506_08481_amd import workloads as wl
    t0 = time.time()
    if args.weights:
        problems = None
        s_test = wl.bidisperse(50000, 0.35, 5000, a1=1.0, a2=2.0)
    else:
        problems = tp.ProblemPool(args.train_configs, 11)      # forked before the GPU is touched
        test_job = problems.pool.apply_async(wl.bidisperse, (50000, 0.35, 5000), dict(a1=1.0, a2=2.0))
    from paper_1506_08481_amd import seasd
    net = seasd.Net(0, seed=11)

    def log(m):
        print(m, file=sys.stderr, flush=True)
    if args.weights:   # the shipped network: no training in this run
        net.load(args.weights)
        hist = []
    else:
        hist = tp.train(net, problems, epochs=args.train_epochs, nrhs=8, lr=5e-4, seed=11, log=log)
    t_train = time.time() - t0
    if args.save_weights:
        net.save(args.save_weights)
    s = s_test if args.weights else test_job.get()
    log(f"trained {len(hist)} steps in {t_train:.0f}s; test N={s.n} L={s.L:.2f}")
    res = tp.evaluate(net, s, tol=1e-6, precision=seasd.SEASD_FP64, repeats=2)
    bd, lg = res["blockdiag"], res["learned_guess"]
    # the same two solves with FP32 products in the Arnoldi steps (FP64 restart residuals)
    rmx = tp.evaluate(net, s, tol=1e-6, precision=seasd.SEASD_MIXED, repeats=2)
    out = {
        "metric": "far-field solve time, learned vs block-diagonal, N=5e4 bidisperse phi=0.35, 1e-6 residual",
        "value": lg["wall_s"], "unit": "s", "higher_is_better": False, "n_gpus": 1,
        "dtype": "f64 product and GMRES, bf16 network",
        "data": "synthetic",
        "config": {"workload": "bidisperse spheres N=50000 (radii 1, 2; equal volume per species) phi=0.35",
                   "N": s.n, "L": s.L, "product": res["config"], "tol": 1e-6, "restart": 50},
        "blockdiag": {k: bd[k] for k in ("iterations", "matvecs", "true_residual", "initial_residual", "wall_s",
                                         "setup_ms")},
        "learned_guess": {k: lg[k] for k in ("iterations", "matvecs", "true_residual", "initial_residual",
                                             "wall_s", "setup_ms", "learned_ms", "guess_used", "guess_scale",
                                             "rel_diff_vs_blockdiag")},
        "iterations_saved": bd["iterations"] - lg["iterations"],
        "speedup_vs_blockdiag": bd["wall_s"] / lg["wall_s"],
        "mixed_precision": {k: {q: rmx[k][q] for q in ("iterations", "true_residual", "wall_s",
                                                      "rel_diff_vs_blockdiag")}
                            for k in ("blockdiag", "learned_guess")},
        "training": ({"weights": args.weights} if args.weights else
                     {"configs": args.train_configs, "epochs": args.train_epochs, "rhs_per_step": 8,
                      "steps": len(hist), "problems_seen": len(hist) * 8,
                      "loss_first_epoch": float(np.mean(hist[:args.train_configs])),
                      "loss_last_epoch": float(np.mean(hist[-args.train_configs:])), "seconds": t_train}),
    }
    print(json.dumps(out), flush=True)


def pmc_probe(args):
    """Three products of the benchmark workload in the given candidate
    configuration, then a 2 GiB fill and three passes c = 2 a over it (torch
    elementwise kernels reading and writing 2 GiB each, far beyond every
    cache), which calibrate the HBM byte counters."""
    import torch

    from paper_1506_08481_amd import seasd
    from paper_1506_08481_amd import workloads as wl
    s = wl.config_large(n=args.n)
    x = wl.force_moments(s.n, 3001)
    dev = torch.device("cuda:0")
    P_, R_, X_ = (torch.as_tensor(a, device=dev) for a in (s.pos, s.radius, x))
    xi, rcf, P, mf = CANDIDATES[args.pmc_candidate]
    eng = seasd.Seasd(0, grid=256, P=P, m=mf * math.sqrt(math.pi * P), xi=xi, rc_factor=rcf,
                      precision=seasd.SEASD_FP32, checks=0)
    y = torch.empty_like(X_)
    for _ in range(3):
        eng.apply(P_, R_, s.box, X_, y)
    a = torch.ones(512 * 1024 * 1024, dtype=torch.float32, device=dev)   # 2 GiB
    c = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 2.0, out=c)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "done", "calibration_bytes_read_and_written": a.numel() * 4}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--workload", choices=["large", "solve", "batch", "learned"], default="large")
    ap.add_argument("--train-configs", type=int, default=96)
    ap.add_argument("--train-epochs", type=int, default=12)
    ap.add_argument("--save-weights", default=None)
    ap.add_argument("--weights", default=None, help="learned workload: use these weights instead of training")
    ap.add_argument("--pmc-probe", action="store_true")
    ap.add_argument("--pmc-candidate", type=int, default=2)
    ap.add_argument("--candidate", type=int, default=None,
                    help="time this candidate without the selection pass (profiling runs)")
    ap.add_argument("--no-solve", action="store_true",
                    help="default workload: skip the learned / block-diagonal solve comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)
    if args.pmc_probe:
        return pmc_probe(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "solve":
        return bench_solve(args)
    if args.workload == "learned":
        return bench_learned(args)

    import torch

    from paper_1506_08481_amd import seasd
    from paper_1506_08481_amd import workloads as wl

    t_setup = time.time()
    s = wl.config_large(n=args.n)
    x = wl.force_moments(s.n, 3001)
    dev = torch.device("cuda:0")
    P_ = torch.as_tensor(s.pos, device=dev)
    R_ = torch.as_tensor(s.radius, device=dev)
    X_ = torch.as_tensor(x, device=dev)
    M = 256
    print(f"setup: N={s.n} L={s.L:.3f} placement {time.time() - t_setup:.1f}s", file=sys.stderr, flush=True)

    def engine(cand, precision):
        xi, rcf, P, mf = cand
        return seasd.Seasd(0, grid=M, P=P, m=mf * math.sqrt(math.pi * P), xi=xi, rc_factor=rcf,
                           precision=precision, checks=0)

    ref_eng = engine(REF, seasd.SEASD_FP64)
    ref_eng.set_config(checks=1)
    yref = ref_eng.apply(P_, R_, s.box, X_).clone()
    ref_eng.close()
    torch.cuda.synchronize()

    # candidate selection: fastest with |y - y_fp64| / |y_fp64| <= 1e-6
    best = None
    tune = []
    for cand in (CANDIDATES if args.candidate is None else [CANDIDATES[args.candidate]]):
        eng = engine(cand, seasd.SEASD_FP32)
        y = eng.apply(P_, R_, s.box, X_)
        torch.cuda.synchronize()
        err = float(torch.linalg.norm(y - yref) / torch.linalg.norm(yref))
        t0 = time.perf_counter()
        for _ in range(5):
            eng.apply(P_, R_, s.box, X_, y)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 5 * 1e3
        tune.append({"xi": cand[0], "rc_factor": cand[1], "P": cand[2],
                     "m": round(cand[3] * math.sqrt(math.pi * cand[2]), 3),
                     "err_vs_fp64": err, "ms": ms})
        print(f"candidate {cand}: err {err:.2e} {ms:.3f} ms", file=sys.stderr, flush=True)
        if err <= 1e-6 and (best is None or ms < best[1]):
            best = (cand, ms, err)
        eng.close()
    if best is None:
        best = (CANDIDATES[-1], None, None)
    cand = best[0]
    eng = engine(cand, seasd.SEASD_FP32)
    y = torch.empty_like(X_)
    for _ in range(args.warmup):
        eng.apply(P_, R_, s.box, X_, y)
    torch.cuda.synchronize()
    eng.profile(True)
    # per-step HIP events on the stream the library queues on (torch's current one)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(args.steps):
        eng.apply(P_, R_, s.box, X_, y)
        ev[k + 1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    phases = eng.profile_read()
    eng.profile(False)
    err = float(torch.linalg.norm(y - yref) / torch.linalg.norm(yref))
    ms_per_step = elapsed / args.steps * 1e3
    eng.close()

    # the plain FP64 method at the same configuration on the same GPU
    eng64 = engine(cand, seasd.SEASD_FP64)
    y64 = torch.empty_like(X_)
    for _ in range(3):
        eng64.apply(P_, R_, s.box, X_, y64)
    torch.cuda.synchronize()
    n64 = max(5, args.steps // 5)
    t0 = time.perf_counter()
    for _ in range(n64):
        eng64.apply(P_, R_, s.box, X_, y64)
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) / n64 * 1e3
    err64 = float(torch.linalg.norm(y64 - yref) / torch.linalg.norm(yref))
    fp32_vs_fp64 = float(torch.linalg.norm(y - y64) / torch.linalg.norm(y64))
    eng64.close()
    # the timed FP32 result against the FP64 oracle at the 2,000 stored
    # target spheres of this workload (written by the oracle alone)
    err_oracle = None
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "large_oracle_sample.npz")
    if args.n == 100000 and os.path.exists(gold):
        d = np.load(gold)
        if np.allclose([s.pos.sum(), (s.pos ** 2).sum()], d["pos_checksum"], rtol=1e-12):
            yc = y.cpu().numpy()[d["targets"]]
            err_oracle = float(np.linalg.norm(yc - d["y"]) / np.linalg.norm(d["y"]))

    pairs = count_pairs(s.pos, s.radius, s.L, cand[1])
    kernel_phases = [k for k in seasd.PHASES if k != "bin"]
    dom = max(kernel_phases, key=lambda k: phases[k])
    cost = phase_cost(dom, s.n, M, cand[2], 4, pairs)
    t_dom = phases[dom] * 1e-3
    if dom == "pair":
        roof = {"bound": "alu", "achieved": cost["flops"] / t_dom / 1e12, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s"}
    elif cost["flops"] / PEAK_FP32_SCALAR_TFLOPS / 1e12 > cost["bytes"] / PEAK_HBM_GBS / 1e9:
        roof = {"bound": "alu", "achieved": cost["flops"] / t_dom / 1e12, "peak": PEAK_FP32_SCALAR_TFLOPS,
                "unit": "TFLOP/s", "peak_note": "FP32 without packed instructions (the published 157.3 "
                                                "counts packed FMAs, which this build does not use)",
                "frac_of_published": cost["flops"] / t_dom / 1e12 / PEAK_FP32_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": cost["bytes"] / t_dom / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = MEASURED_TRAFFIC.get((dom, M, cand[2]))
    roof["kernel"] = dom
    roof["kernel_ms"] = phases[dom]

    out = {
        "metric": "M·F matvecs/s at N=1e5, φ=0.4, 1e-6 err; solve time learned vs block-diag",
        "value": 1e3 / ms_per_step,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "monodisperse spheres N=100000 phi=0.4, grid 256^3, FP32 spread/FFT/gather, "
                               "FP64 pair sum", "N": s.n, "L": s.L, "grid": M,
                   "xi": cand[0], "rc_factor": cand[1], "P": cand[2],
                   "m": cand[3] * math.sqrt(math.pi * cand[2])},
        "rel_err_vs_fp64_gpu": err,
        "rel_err_vs_oracle_2000_targets": err_oracle,
        "step_ms": {"median": float(np.median(step_ms)), "p10": float(np.percentile(step_ms, 10)),
                    "p90": float(np.percentile(step_ms, 90))},
        "matvecs_per_s_median": 1e3 / float(np.median(step_ms)),
        "fp64_same_config": {"matvecs_per_s": 1e3 / ms64, "ms_per_step": ms64, "steps": n64,
                             "rel_err_vs_fp64_reference": err64,
                             "fp32_minus_fp64_rel": fp32_vs_fp64,
                             "speedup_fp32": ms64 / ms_per_step},
        "phases_ms": {k: round(v, 5) for k, v in phases.items()},
        "tuning": tune,
        "roofline": roof,
    }
    if args.candidate is None and not args.no_solve:
        # the second half of the metric; the product figures above stand on
        # their own if it fails, and the failure is reported in its place
        try:
            out["solve_learned_vs_blockdiag"] = learned_vs_blockdiag()
        except Exception as e:  # noqa: BLE001
            out["solve_learned_vs_blockdiag"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, x)
    print(json.dumps(out))


def learned_vs_blockdiag():
    """The shipped network against the block-diagonal preconditioner alone on
    the learned-preconditioner test suspension (N = 50,000 bidisperse, radii 1
    and 2, phi = 0.35, never seen in training), far-field GMRES(50) to a true
    residual of 1e-6: FP64 products, and FP32 products in the Arnoldi steps
    (precision SEASD_MIXED)."""
    from paper_1506_08481_amd import seasd
    from paper_1506_08481_amd import train_precond as tp
    from paper_1506_08481_amd import workloads as wl
    weights = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1506_08481_amd", "weights",
                           "precond_mpnn.bin")
    s = wl.bidisperse(50000, 0.35, 5000, a1=1.0, a2=2.0)
    net = seasd.Net(0, seed=11)
    net.load(weights)
    out = {"workload": "bidisperse N=50000 (radii 1, 2) phi=0.35, tol 1e-6, GMRES(50), shipped network"}
    for key, prec in (("fp64", seasd.SEASD_FP64), ("mixed_precision", seasd.SEASD_MIXED)):
        r = tp.evaluate(net, s, tol=1e-6, precision=prec, repeats=1)
        bd, lg = r["blockdiag"], r["learned_guess"]
        out[key] = {"blockdiag_s": bd["wall_s"], "learned_s": lg["wall_s"],
                    "blockdiag_iterations": bd["iterations"], "learned_iterations": lg["iterations"],
                    "learned_true_residual": lg["true_residual"], "network_ms": lg["learned_ms"],
                    "speedup_learned": bd["wall_s"] / lg["wall_s"]}
    net.close()
    return out


if __name__ == "__main__":
    main()
