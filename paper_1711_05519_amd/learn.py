"""Training of the learned threshold schedule (an extension; the paper fixes
zeta_{k+1} = beta (sigma_{r+1} + gamma^{k+1} sigma_1), Algorithm 1).

The network maps features of the iterate to a correction of the paper's
threshold, zeta_k = zeta_paper,k * exp(clip(o_k, -5, 5)) (see include/rpca.h,
RPCA_FLAG_LEARNED); the untrained network (zero output layer) reproduces the
paper's schedule. It is trained on synthetic instances with known ground
truth L = P Q^T by unrolling `steps` iterations with the relaxed threshold
s(x) = x * logistic((|x| - zeta) / tau); the objective is the mean of
log ||L_{k+1} - L||_F^2 / ||L||_F^2 over the iterations whose threshold came
from the network (k >= 1). Two ways of differentiating it:

* mode "unrolled": through all unrolled iterations (rpca_unrolled_adjoint,
  from factor checkpoints): d/dzeta_k of sum_j w_j loss_j with w_j =
  1 / loss_j (the gradient of sum_j log loss_j), so a threshold is credited
  with its effect on every later iterate;
* mode "one": one step at a time (the derivative of rpca_relaxed_step): the
  state reached is data for the next step, zeta_k sees only loss_{k+1}.

Either way d zeta_k / d o_k = zeta_k inside the clip, the features are held
fixed, and the network's backward kernel and Adam update the parameters.
tau is annealed as tau_e = tau0 * 0.5^e (relative to zeta). The passes over D,
the relaxed iterations, the adjoints and the network's forward, backward and
Adam update run in the library's kernels; this module sequences the calls and
does the scalar bookkeeping on the host between them (Algorithm 1's threshold
for the next step from the sigma values a step returns, the clip of the
correction and the chain rule to o, a few flops per step).
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import inputs as I
from . import rpca as R

K_FEAT = 15.0       # normalises the iteration index in the features
FEATURE_FLOOR = 1e-30
SIGMA_RATIO_FLOOR = 1e-4   # sigma_{r+1} / sigma_1 below this is rounding noise in the FP32 path
# The loss is formed from inner products in the reduced space, so below about
# 1e-12 it is at the rounding level of ||L||_F^2: such steps carry no signal.
LOSS_FLOOR = 1e-12


def features(k: int, sigma1: float, sigma_r1: float, err: float, normD: float) -> list[float]:
    """phi = (k / 15, log max(sigma_{r+1} / sigma_1, 1e-4), log err, log(sigma_1 / ||D||_F)) for choosing zeta_k."""
    f = FEATURE_FLOOR
    return [k / K_FEAT, math.log(max(sigma_r1 / max(sigma1, f), SIGMA_RATIO_FLOOR)), math.log(max(err, f)),
            math.log(max(sigma1, f) / max(normD, f))]


O_CLIP = 5.0


def init_theta(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-style hidden weights, zero biases and a zero output layer: the
    untrained network outputs o = 0, i.e. the paper's schedule."""
    g = np.random.default_rng(seed)
    W1 = g.standard_normal((32, 4)) * math.sqrt(2.0 / 4)
    W2 = g.standard_normal((32, 32)) * math.sqrt(2.0 / 32)
    th = np.concatenate([W1.ravel(), np.zeros(32), W2.ravel(), np.zeros(32), np.zeros(32), [0.0]])
    return torch.tensor(th, dtype=torch.float32, device=device)


def save_theta(theta: torch.Tensor, path: str) -> None:
    np.save(path, theta.detach().cpu().numpy().astype(np.float32), allow_pickle=False)


def load_theta(path: str, device="cuda") -> torch.Tensor:
    a = np.load(path, allow_pickle=False)
    if a.shape != (R.RPCA_MLP_PARAMS,):
        raise ValueError(f"{path}: expected {R.RPCA_MLP_PARAMS} parameters")
    return torch.tensor(a, dtype=torch.float32, device=device)


@dataclasses.dataclass
class Problem:
    solver: R.Solver
    P: torch.Tensor
    Q: torch.Tensor
    beta: float
    start: tuple          # state after rpca_init


def make_problem(x: I.Instance, dtype=torch.float64, device="cuda") -> Problem:
    D = torch.as_tensor(x.D, dtype=dtype, device=device)
    sv = R.Solver(D, x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol, training=True, seed=1)
    sv.init()
    return Problem(sv, torch.as_tensor(x.P, dtype=torch.float64, device=device),
                   torch.as_tensor(x.Q, dtype=torch.float64, device=device), x.beta, sv.get_state())


def unroll(pb: Problem, theta: torch.Tensor | None, steps: int, tau_rel: float):
    """Unrolled relaxed iterations from the initial state. zeta_0 is the
    initialisation's; zeta_k (k >= 1) comes from the network (theta) or, with
    theta None, from the paper's schedule. Returns the per-step losses and, for
    training, the features and d log loss / d o of every network call."""
    sv = pb.solver
    sv.put_state(pb.start)
    normD = sv.state.normD
    zeta = sv.state.zeta
    res = sv.relaxed_step(zeta, tau_rel * zeta, pb.P, pb.Q)
    losses = [res.loss]
    phis, gos = [], []
    for k in range(1, steps):
        zeta = pb.beta * (res.sigma_r1 + sv.params.gamma ** k * res.sigma1)   # Algorithm 1
        inside = True
        if theta is not None:
            phi = torch.tensor([features(k, res.sigma1, res.sigma_r1, res.err, normD)], dtype=torch.float32,
                               device=theta.device)
            o = float(R.rpca_mlp_forward(theta, phi)[0])
            inside = -O_CLIP < o < O_CLIP
            zeta *= math.exp(min(max(o, -O_CLIP), O_CLIP))
        res = sv.relaxed_step(zeta, tau_rel * zeta, pb.P, pb.Q)
        losses.append(res.loss)
        if theta is not None and res.loss > LOSS_FLOOR and math.isfinite(res.dloss_dzeta):
            phis.append(phi[0])
            # d log loss / d o = (d loss / d zeta) zeta / loss inside the clip
            gos.append(res.dloss_dzeta * zeta / res.loss if inside else 0.0)
    return losses, phis, gos


def unroll_full(pb: Problem, theta: torch.Tensor, steps: int, tau_rel: float):
    """As unroll, keeping the factor checkpoints, and the gradient of the
    mean log loss of the iterations k >= 1 through all of them: returns the
    per-step losses, the features and d objective / d o of every network call."""
    sv = pb.solver
    sv.put_state(pb.start)
    normD = sv.state.normD
    zetas, taus, losses, phis, inside = [], [], [], [], []
    zeta = sv.state.zeta
    res = None
    for k in range(steps):
        if k >= 1:
            zeta = pb.beta * (res.sigma_r1 + sv.params.gamma ** k * res.sigma1)   # Algorithm 1
            phi = torch.tensor([features(k, res.sigma1, res.sigma_r1, res.err, normD)], dtype=torch.float32,
                               device=theta.device)
            o = float(R.rpca_mlp_forward(theta, phi)[0])
            inside.append(-O_CLIP < o < O_CLIP)
            zeta *= math.exp(min(max(o, -O_CLIP), O_CLIP))
            phis.append(phi[0])
        zetas.append(zeta)
        taus.append(tau_rel * zeta)
        if k == 0:
            ck = [(sv.U.clone(), sv.sigma.clone(), sv.V.clone())]
        res = sv.relaxed_step(zeta, tau_rel * zeta, pb.P, pb.Q)
        losses.append(res.loss)
        ck.append((sv.U.clone(), sv.sigma.clone(), sv.V.clone()))
    # weights of loss_{k+1} = ||L_{k+1} - L||^2 / ||L||^2: 1 / loss for the network's steps
    use = [k >= 1 and losses[k] > LOSS_FLOOR for k in range(steps)]
    cnt = max(sum(use), 1)
    w = [(1.0 / losses[k]) / cnt if use[k] else 0.0 for k in range(steps)]
    if not any(use):
        return losses, [], []
    zb, _, _, _ = sv.unrolled_adjoint(ck, zetas, taus, w, pb.P, pb.Q)
    if not np.all(np.isfinite(zb)):
        return losses, [], []
    gos = [float(zb[k]) * zetas[k] if inside[k - 1] else 0.0 for k in range(1, steps)]
    return losses, phis, gos


VALIDATION_IDS = (500, 501, 502, 503)   # training pool instances held out of the training set (small runs)
POOL = 512                              # instances 0 .. 511 form the training pool, 512 .. 575 the test set


def split(n_instances: int):
    """Gradient instances and validation instances of a run on the first
    n_instances of the pool: runs on the whole pool keep its last 32 for
    choosing the epoch; smaller runs validate on VALIDATION_IDS."""
    if n_instances >= 256:
        return list(range(n_instances - 32)), tuple(range(n_instances - 32, n_instances))
    return list(range(n_instances)), VALIDATION_IDS


_SOLVE_CACHE: dict = {}   # (instance, dtype) -> (instance without D, D on the device)


def _instance_on_device(i: int, dtype):
    key = (i, dtype)
    if key not in _SOLVE_CACHE:
        x = I.config_instance(5, i, keep_L=False)
        D = torch.as_tensor(x.D, dtype=dtype, device="cuda")
        x.D = None
        _SOLVE_CACHE[key] = (x, D)
    return _SOLVE_CACHE[key]


def solve_stats(theta, ids, dtype=torch.float32):
    """Real (hard-threshold) solves to tol: (mean iterations, worst recovery
    error ||L - L_true||_F / ||L_true||_F, all converged)."""
    its, worst, ok = [], 0.0, True
    for i in ids:
        x, D = _instance_on_device(i, dtype)
        sv = R.Solver(D, x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol, seed=1, learned=theta)
        info = sv.solve()
        U, s_, V = sv.L_factors()
        P = torch.as_tensor(x.P, dtype=torch.float64, device="cuda")
        Q = torch.as_tensor(x.Q, dtype=torch.float64, device="cuda")
        # ||U S V^T - P Q^T||_F^2 from r x r products (no dense matrix)
        a = (U * s_).T @ (U * s_)
        b = V.T @ V
        c = P.T @ P
        d = Q.T @ Q
        cross = ((U * s_).T @ P) * (V.T @ Q)
        num = float((a * b).sum() - 2.0 * cross.sum() + (c * d).sum())
        rec = math.sqrt(max(num, 0.0) / float((c * d).sum()))
        its.append(info.iterations)
        worst = max(worst, rec)
        ok = ok and info.status == R.RPCA_OK
    return sum(its) / len(its), worst, ok


def train(n_instances: int = 32, epochs: int = 12, steps: int = 15, tau0: float = 0.2, lr: float = 3e-4,
          seed: int = 0, dtype=torch.float64, log=print, mode: str = "one"):
    """Trains the network (mode "one" or "unrolled", see the module
    docstring) on the first n_instances of the training pool
    (inputs.config_instance(5, i)), split into gradient and validation
    instances (split()). After every epoch the network solves the validation
    instances to tol with the hard threshold; the returned theta is the epoch
    with the fewest mean iterations among those whose solves all converge with
    recovery error <= 1e-4 (the untrained network, i.e. the paper's schedule,
    if none). Returns (theta, history)."""
    dev = torch.device("cuda")
    t0 = time.perf_counter()
    train_ids, val_ids = split(n_instances)
    problems = []
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=8) as ex:   # instance draws on the host, in parallel
        for x in ex.map(lambda i: I.config_instance(5, i, keep_L=False), train_ids):
            problems.append(make_problem(x, dtype, dev))
            if len(problems) % 64 == 0:
                log(f"{len(problems)} of {len(train_ids)} training instances ready ({time.perf_counter() - t0:.1f} s)")
    log(f"{len(train_ids)} training instances ready in {time.perf_counter() - t0:.1f} s; "
        f"validation on {len(val_ids)} instances")
    theta = init_theta(seed, dev)
    best = theta.clone()
    best_its, _, _ = solve_stats(None, val_ids)
    log(f"paper schedule: {best_its:.2f} mean iterations on the validation instances")
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    t = 0
    hist = []
    for e in range(epochs):
        tau_rel = tau0 * 0.5 ** e
        tot, cnt = 0.0, 0
        for pb in problems:
            if mode == "unrolled":
                losses, phis, gos = unroll_full(pb, theta, steps, tau_rel)
            else:
                losses, phis, gos = unroll(pb, theta, steps, tau_rel)
            tot += sum(math.log(max(l, LOSS_FLOOR)) for l in losses[1:])
            cnt += len(losses) - 1
            if not phis:
                continue
            phi = torch.stack(phis).contiguous()
            # "one": mean over the steps of d log loss_{k+1} / d o_k; "unrolled": already the mean
            g = torch.tensor(gos, dtype=torch.float32, device=dev) / (len(gos) if mode != "unrolled" else 1)
            grad = R.rpca_mlp_backward(theta, phi, g)
            t += 1
            R.rpca_mlp_adam(theta, m, v, grad, t, lr)
        hist.append(tot / max(cnt, 1))
        its, rec, ok = solve_stats(theta, val_ids)
        keep = ok and rec <= 1e-4 and its < best_its
        if keep:
            best, best_its = theta.clone(), its
        log(f"epoch {e}: tau/zeta {tau_rel:.4f}  mean log loss {hist[-1]:.4f}  validation: {its:.2f} it, "
            f"recovery {rec:.1e}{'  (kept)' if keep else ''}  ({time.perf_counter() - t0:.1f} s)")
    train.last = theta.clone()   # the final epoch's parameters, kept or not
    return best, hist


def evaluate(theta: torch.Tensor | None, ids, steps: int = 15, tau_rel: float = 1e-6, dtype=torch.float64):
    """Mean log loss of the unrolled iterations on instances ids of the pool."""
    tot, cnt = 0.0, 0
    for i in ids:
        pb = make_problem(I.config_instance(5, i), dtype)
        losses, _, _ = unroll(pb, theta, steps, tau_rel)
        tot += sum(math.log(max(l, LOSS_FLOOR)) for l in losses[1:])
        cnt += len(losses) - 1
    return tot / max(cnt, 1)


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="train the learned threshold network")
    ap.add_argument("--instances", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--steps", type=int, default=15)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--test", type=int, default=64, help="held-out test instances 512, 513, ... after training")
    ap.add_argument("--compare", default="", help="another parameter file to evaluate on the test instances")
    ap.add_argument("--mode", choices=["one", "unrolled"], default="one",
                    help="differentiate one step at a time or through all unrolled iterations")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    ap2_test = list(range(POOL, POOL + a.test))
    th, hist = train(a.instances, a.epochs, a.steps, lr=a.lr, mode=a.mode)
    save_theta(th, a.out)
    save_theta(train.last, a.out.replace(".npy", "") + "_last.npy")
    print(f"held-out mean log loss (first 8): paper {evaluate(None, ap2_test[:8], a.steps):.4f}  "
          f"learned {evaluate(th, ap2_test[:8], a.steps):.4f}", flush=True)
    # real (hard-threshold) solves on the held-out test instances
    others = [("compared", load_theta(a.compare))] if a.compare else []
    for name, theta in [("paper", None), ("learned (selected epoch)", th), ("learned (last epoch)", train.last)] + others:
        its, rec, ok = solve_stats(theta, ap2_test)
        print(f"held-out solves ({len(ap2_test)} instances {ap2_test[0]}..{ap2_test[-1]}), {name}: {its:.3f} mean "
              f"iterations, worst recovery {rec:.1e}, all converged {ok}", flush=True)
