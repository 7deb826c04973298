"""Reverse mode of unrolled relaxed iterations (rpca_unrolled_adjoint) against
the FP64 oracle (oracle/adjoint.py, pinned by central differences): the
thresholds' gradients and the gradients of the initial factors, over several
bodies, with and without Trim, across several column and row tiles with
ragged edges; plus the autograd Function and central differences of the
library's own forward."""
import sys

import numpy as np
import pytest
import torch

from oracle import accaltproj as A
from oracle import adjoint as J
from paper_1711_05519_amd import rpca as R

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def instance(m, n, r, alpha, seed, mu, dtype):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((m, r))
    Q = rng.standard_normal((n, r))
    T = P @ Q.T
    S = np.zeros((m, n))
    sup = rng.random((m, n)) < alpha
    S[sup] = rng.uniform(-1.0, 1.0, sup.sum()) * 2.0 * np.mean(np.abs(T))
    D = T + S
    if dtype == torch.float32:
        D = D.astype(np.float32).astype(np.float64)
    U0, s0, V0 = A.best_rank_r(T + 0.3 * rng.standard_normal((m, n)), r)
    p = A.Params(r=r, beta=0.5, beta_init=1.0, gamma=0.6, mu=mu)
    return D, P, Q, U0, s0, V0, p


def gpu_adjoint(D, P, Q, U0, s0, V0, p, zetas, taus, w, dtype):
    sv = R.Solver(dev(D, dtype), p.r, p.beta, p.beta_init, p.gamma, p.mu if p.mu > 0 else 1.0,
                  trim=p.mu > 0, training=True)
    sv.set_state(U0, s0, V0, zetas[0], 0)
    Pd, Qd = dev(P), dev(Q)
    losses, ck = sv.unrolled(zetas, taus, w, Pd, Qd)
    zb, Ub, sb, Vb = sv.unrolled_adjoint(ck, zetas, taus, w, Pd, Qd)
    return losses, zb, Ub.cpu().numpy(), sb.cpu().numpy(), Vb.cpu().numpy()


CASES = [
    # m, n, r, alpha, mu, K
    (150, 130, 3, 0.1, 1.5, 4),
    (150, 130, 3, 0.1, 0.0, 4),
    (700, 600, 5, 0.1, 2.0, 3),
    (300, 520, 2, 0.05, 1.5, 1),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_unrolled_adjoint_matches_oracle(case, dtype):
    m, n, r, alpha, mu, K = case
    say(f"unrolled adjoint m={m} n={n} r={r} mu={mu} K={K} {dtype}")
    D, P, Q, U0, s0, V0, p = instance(m, n, r, alpha, 7 + m + K, mu, dtype)
    T = P @ Q.T
    zetas = [0.9 * float(np.max(np.abs(T))) * 0.6 ** k for k in range(K)]
    taus = [0.2 * z for z in zetas]
    w = [0.5 + 0.5 * k for k in range(K)]
    if mu > 0:
        cU, cV = J.trim_levels(m, n, mu, r)
        assert np.any(np.linalg.norm(U0, axis=1) > cU) or np.any(np.linalg.norm(V0, axis=1) > cV)
    losses, zb, Ub, sb, Vb = gpu_adjoint(D, P, Q, U0, s0, V0, p, zetas, taus, w, dtype)
    ref = J.unrolled_adjoint(D, U0, s0, V0, zetas, taus, w, p, P, Q)
    errs = (rel(losses, ref.losses), rel(zb, ref.zeta_bar), rel(Ub, ref.Ubar0), rel(sb, ref.sbar0), rel(Vb, ref.Vbar0))
    say("  rel. differences: losses %.2e  dzeta %.2e  dU0 %.2e  dsigma0 %.2e  dV0 %.2e" % errs)
    # FP64: the same algebra in another order; FP32: the relaxed forward
    # rounds D and its factor copies to FP32 (relative 6e-8), which the
    # gradients see amplified by the conditioning of the iterations
    tol = 1e-8 if dtype == torch.float64 else 2e-4
    assert max(errs) < tol, errs


def test_autograd_function_and_forward_differences():
    m, n, r, K = 200, 180, 3, 3
    D, P, Q, U0, s0, V0, p = instance(m, n, r, 0.1, 99, 1.5, torch.float64)
    T = P @ Q.T
    zetas = [0.9 * float(np.max(np.abs(T))) * 0.6 ** k for k in range(K)]
    taus = [0.2 * z for z in zetas]
    w = [0.25, 0.5, 1.0]
    sv = R.Solver(dev(D), r, p.beta, p.beta_init, p.gamma, p.mu, training=True)
    Pd, Qd = dev(P), dev(Q)
    z = torch.tensor(zetas, dtype=torch.float64, device="cuda", requires_grad=True)
    U = dev(U0).requires_grad_(True)
    s = dev(s0).requires_grad_(True)
    V = dev(V0).requires_grad_(True)
    loss = R.UnrolledRelaxed.apply(z, U, s, V, sv, Pd, Qd, taus, w)
    loss.backward()
    ref = J.unrolled_adjoint(D, U0, s0, V0, zetas, taus, w, p, P, Q)
    assert abs(float(loss) - ref.loss) <= 1e-10 * ref.loss
    assert rel(z.grad.cpu().numpy(), ref.zeta_bar) < 1e-8
    assert rel(U.grad.cpu().numpy(), ref.Ubar0) < 1e-8
    assert rel(s.grad.cpu().numpy(), ref.sbar0) < 1e-8
    assert rel(V.grad.cpu().numpy(), ref.Vbar0) < 1e-8

    # central differences of the library's forward in each threshold
    def f(k, h):
        zz = list(zetas)
        zz[k] += h
        sv.set_state(U0, s0, V0, zz[0], 0)
        losses, _ = sv.unrolled(zz, taus, w, Pd, Qd)
        return sum(a * b for a, b in zip(w, losses))

    for k in range(K):
        h = 1e-5 * zetas[k]
        num = (f(k, h) - f(k, -h)) / (2 * h)
        say(f"  k={k}: d loss / d zeta_k adjoint {float(z.grad[k]):.6e}, central difference {num:.6e}")
        assert abs(num - float(z.grad[k])) <= 1e-5 * np.max(np.abs(ref.zeta_bar))


def test_adjoint_rejects_bad_arguments():
    D, P, Q, U0, s0, V0, p = instance(64, 60, 2, 0.1, 1, 1.5, torch.float64)
    sv = R.Solver(dev(D), 2, p.beta, p.beta_init, p.gamma, p.mu, training=True)
    ck = [(dev(U0), dev(s0), dev(V0))] * 2
    Pd, Qd = dev(P), dev(Q)
    with pytest.raises(R.RpcaError):
        sv.unrolled_adjoint(ck, [-1.0], [0.1], [1.0], Pd, Qd)    # zeta <= 0
    with pytest.raises(R.RpcaError):
        sv.unrolled_adjoint(ck, [1.0], [0.0], [1.0], Pd, Qd)     # tau <= 0
    plain = R.Solver(dev(D), 2, p.beta, p.beta_init, p.gamma, p.mu)
    with pytest.raises(R.RpcaError):
        plain.unrolled_adjoint(ck, [1.0], [0.1], [1.0], Pd, Qd)  # no training workspace


def test_unrolled_adjoint_at_the_limits():
    """r = 10 (the largest rank of the relaxed iteration), a target of rank 16
    and K = 15 unrolled bodies, FP64, against the oracle."""
    m, n, r, K = 260, 240, 10, 15
    rng = np.random.default_rng(5)
    D, P0, Q0, U0, s0, V0, p = instance(m, n, r, 0.05, 9, 2.0, torch.float64)
    # a target of rank 16: the true factors plus six small extra directions
    P = np.hstack([P0, 1e-2 * rng.standard_normal((m, 6))])
    Q = np.hstack([Q0, 1e-2 * rng.standard_normal((n, 6))])
    T = P0 @ Q0.T
    zetas = [0.9 * float(np.max(np.abs(T))) * 0.7 ** k for k in range(K)]
    taus = [0.2 * z for z in zetas]
    w = [1.0 / K] * K
    losses, zb, Ub, sb, Vb = gpu_adjoint(D, P, Q, U0, s0, V0, p, zetas, taus, w, torch.float64)
    ref = J.unrolled_adjoint(D, U0, s0, V0, zetas, taus, w, p, P, Q)
    errs = (rel(losses, ref.losses), rel(zb, ref.zeta_bar), rel(Ub, ref.Ubar0), rel(sb, ref.sbar0), rel(Vb, ref.Vbar0))
    say("  r=10 rt=16 K=15: losses %.2e  dzeta %.2e  dU0 %.2e  dsigma0 %.2e  dV0 %.2e" % errs)
    assert max(errs) < 1e-7, errs
