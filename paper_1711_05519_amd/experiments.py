"""The synthetic-data experiments of Section 3 on one GPU (runtimes of the
library's solver; the comparison systems are not part of this package).

  python -m paper_1711_05519_amd.experiments table2 [--trials 10]
      Table 2: rate of success of AccAltProj with and without trim, n = 2500,
      r = 5, tol 1e-6, at most 100 iterations, c in {0.2, 1, 5},
      alpha = 0.30 .. 0.75; success when ||L_k - L||_F / ||L||_F <= 1e-4. FP64.
  python -m paper_1711_05519_amd.experiments nsweep
      Figure 2(a): time to err_k < 1e-4 against n = 1000 .. 15000 (r = 5,
      alpha = 0.1, c = 1), FP32 and FP64 D.
  python -m paper_1711_05519_amd.experiments alphasweep
      Figure 2(b): time to err_k < 1e-4 or 100 iterations against alpha
      (r = 5, c = 1, n = 2500), FP64.
  python -m paper_1711_05519_amd.experiments errtime
      Figure 2(c): err_k against the time to reach iteration k (r = 5,
      alpha = 0.1, c = 1, n = 2500, stop at err_k < 1e-5), FP64 and FP32.
  python -m paper_1711_05519_amd.experiments many [--count 32]
      Throughput on many small problems (the instance pool of the learned
      threshold: 2000 x 2000, r = 5 .. 10, alpha 0.05 .. 0.3, FP32): solves
      one after another against rpca_solve_many on 4, 8 and 16 streams and
      against rpca_solve_batch (one batch per rank, every launch covering
      all instances of the batch), one batch after another and on 3 streams.
  python -m paper_1711_05519_amd.experiments video
      Video-shaped workload (144 x 176 pixels x 2000 frames, r = 2, the
      stand-in for the background-subtraction data): time, iterations and the
      incoherence of the output L with and without trim, FP32.

Inputs are the seeded synthetic instances of inputs.py; times are seconds per
solve with D resident in device memory (median of --reps timed solves after
one warm-up). Each result is printed as one JSON line.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import time

import numpy as np
import torch

from . import inputs as I
from . import rpca as R

CONFIG_ID = 30   # seeds of these experiments: inputs.seed_for(30 + experiment, instance)


def emit(**kw):
    print(json.dumps(kw), flush=True)


def timed_solve(sv: R.Solver, reps: int):
    sv.solve()                      # warm-up
    torch.cuda.synchronize()
    ts = []
    info = None
    for _ in range(reps):
        t0 = time.perf_counter()
        info = sv.solve()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), info


def recovery(sv: R.Solver, x: I.Instance) -> float:
    """||L_k - P Q^T||_F / ||P Q^T||_F from r x r products."""
    U, s, V = (t.cpu().numpy() for t in sv.L_factors())
    a = (U * s).T @ (U * s) * (V.T @ V)
    c = ((U * s).T @ x.P) * (V.T @ x.Q)
    b = (x.P.T @ x.P) * (x.Q.T @ x.Q)
    return math.sqrt(max(a.sum() + b.sum() - 2.0 * c.sum(), 0.0) / b.sum())


def incoherence(sv: R.Solver) -> float:
    """mu of the output L_k = U diag(sigma) V^T (U, V orthonormal)."""
    U, _, V = (t.cpu().numpy() for t in sv.L_factors())
    m, r = U.shape
    n = V.shape[0]
    return max(m / r * float(np.max(np.sum(U * U, axis=1))), n / r * float(np.max(np.sum(V * V, axis=1))))


def solver(x: I.Instance, dtype, tol, max_iter=100, trim=True):
    D = torch.as_tensor(x.D, dtype=dtype, device="cuda")
    return R.Solver(D, x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=tol, max_iter=max_iter, trim=trim, seed=1)


def table2(args):
    alphas = [0.3, 0.35, 0.4, 0.45, 0.5, 0.55, 0.6, 0.65, 0.7, 0.75]
    for c in (0.2, 1.0, 5.0):
        for a in alphas:
            wins = {"with_trim": 0, "without_trim": 0}
            for t in range(args.trials):
                x = I.gaussian_instance(2500, 2500, 5, a, c, tol=1e-6,
                                        seed=I.seed_for(CONFIG_ID + 1, 10000 * int(10 * c) + 100 * int(round(100 * a)) + t))
                for name, trim in (("with_trim", True), ("without_trim", False)):
                    sv = solver(x, torch.float64, 1e-6, trim=trim)
                    sv.solve()
                    wins[name] += int(recovery(sv, x) <= 1e-4)
            emit(experiment="table2", c=c, alpha=a, trials=args.trials, **wins)


def nsweep(args):
    for n in (1000, 2500, 5000, 7500, 10000, 12500, 15000):
        x = I.gaussian_instance(n, n, 5, 0.1, 1.0, tol=1e-4, seed=I.seed_for(CONFIG_ID + 2, n))
        for dtype, name in ((torch.float32, "f32"), (torch.float64, "f64")):
            sv = solver(x, dtype, 1e-4)
            s, info = timed_solve(sv, args.reps)
            emit(experiment="nsweep", n=n, dtype=name, seconds=s, iterations=info.iterations,
                 init_passes=info.init_passes, err=info.err, recovery=recovery(sv, x))
            del sv
        del x
        torch.cuda.empty_cache()


def alphasweep(args):
    for a in (0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4, 0.45, 0.5, 0.55, 0.6, 0.65, 0.7):
        x = I.gaussian_instance(2500, 2500, 5, a, 1.0, tol=1e-4, seed=I.seed_for(CONFIG_ID + 3, int(round(100 * a))))
        sv = solver(x, torch.float64, 1e-4, max_iter=100)
        s, info = timed_solve(sv, args.reps)
        emit(experiment="alphasweep", alpha=a, seconds=s, iterations=info.iterations, status=info.status,
             err=info.err, recovery=recovery(sv, x))


def errtime(args):
    x = I.gaussian_instance(2500, 2500, 5, 0.1, 1.0, tol=1e-5, seed=I.seed_for(CONFIG_ID + 4, 0))
    for dtype, name in ((torch.float64, "f64"), (torch.float32, "f32")):
        full = solver(x, dtype, 1e-5)
        info = full.solve()
        for k in range(0, info.iterations + 1):
            sv = solver(x, dtype, 1e-5, max_iter=k)   # stops at err_k < tol or after k bodies
            s, ik = timed_solve(sv, args.reps)
            emit(experiment="errtime", dtype=name, k=k, seconds=s, err=ik.err)


def many(args):
    # the timed regions run with Python's collector held off (a collection of
    # the host-side objects would otherwise land inside one of them)
    xs = [I.config_instance(5, i, keep_L=False) for i in range(args.count)]
    Ds = [torch.as_tensor(x.D, dtype=torch.float32, device="cuda") for x in xs]

    def solvers():
        return [R.Solver(D, x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol, seed=1) for x, D in zip(xs, Ds)]

    svs = solvers()
    for sv in svs:          # warm-up
        sv.solve()
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    its = [sv.solve().iterations for sv in svs]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    gc.enable()
    emit(experiment="many", mode="one by one", count=args.count, seconds=t_seq, per_solve=t_seq / args.count,
         iterations=sum(its))
    for ns in (4, 8, 16):
        svs = solvers()
        R.solve_many(svs, n_streams=ns)     # warm-up
        torch.cuda.synchronize()
        gc.collect()
        gc.disable()
        t0 = time.perf_counter()
        infos = R.solve_many(svs, n_streams=ns)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        gc.enable()
        emit(experiment="many", mode=f"{ns} streams", count=args.count, seconds=t, per_solve=t / args.count,
             iterations=sum(i.iterations for i in infos), speedup=t_seq / t,
             same_iterations=[i.iterations for i in infos] == its)
    # batched: one rpca_solve_batch per rank r (every kernel launch covers the
    # instances of that rank); D is copied into the slabs before timing
    groups = {}
    for i, x in enumerate(xs):
        groups.setdefault(x.r, []).append(i)
    batches = []
    for r, idx in sorted(groups.items()):
        gx = [xs[i] for i in idx]
        bs = R.BatchSolver(torch.stack([Ds[i] for i in idx]), r, [x.beta for x in gx], [x.beta_init for x in gx],
                           [x.gamma for x in gx], [x.mu_in for x in gx], tol=[x.tol for x in gx], seed=1)
        batches.append((idx, bs))
    for _, bs in batches:   # warm-up
        bs.solve()
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    res = [(idx, bs.solve()) for idx, bs in batches]
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    gc.enable()
    its_b = [0] * args.count
    for idx, infos in res:
        for i, info in zip(idx, infos):
            its_b[i] = info.iterations
    emit(experiment="many", mode=f"batched ({len(batches)} batches, one per rank)", count=args.count,
         seconds=t, per_solve=t / args.count, iterations=sum(its_b), speedup=t_seq / t, same_iterations=its_b == its,
         bytes_of_D=args.count * xs[0].m * xs[0].n * 4)
    # the same batches on 3 streams from 3 host threads (solve_batches)
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    res = R.solve_batches([bs for _, bs in batches], n_streams=3)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    gc.enable()
    its_c = [0] * args.count
    for (idx, _), infos in zip(batches, res):
        for i, info in zip(idx, infos):
            its_c[i] = info.iterations
    emit(experiment="many", mode=f"batched ({len(batches)} batches) on 3 streams", count=args.count,
         seconds=t, per_solve=t / args.count, iterations=sum(its_c), speedup=t_seq / t, same_iterations=its_c == its,
         bytes_of_D=args.count * xs[0].m * xs[0].n * 4)


def video(args):
    x = I.config_instance(3, keep_L=False)
    for trim in (True, False):
        sv = solver(x, torch.float32, x.tol, trim=trim)
        s, info = timed_solve(sv, args.reps)
        emit(experiment="video", m=x.m, n=x.n, r=x.r, trim=trim, seconds=s, iterations=info.iterations,
             err=info.err, recovery=recovery(sv, x), mu_out=incoherence(sv), mu_true=x.mu)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("what", choices=["table2", "nsweep", "alphasweep", "errtime", "video", "many", "all"])
    ap.add_argument("--count", type=int, default=32)
    ap.add_argument("--trials", type=int, default=10)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    todo = ["nsweep", "alphasweep", "errtime", "video", "many", "table2"] if args.what == "all" else [args.what]
    for w in todo:
        globals()[w](args)


if __name__ == "__main__":
    main()
