"""Relaxed iteration and its hand-written zeta-adjoint (rpca_relaxed_step)
against the FP64 oracle of the learned-threshold extension.

Parity unpinned by the paper (it has no relaxed threshold); the oracle used
here is itself pinned by central finite differences and limits in
tests/test_oracle_learned.py. Bars: FP64 loss and next iterate to 1e-9, the
derivative to 1e-7 relative; FP32 data to 1e-4; and the GPU derivative against
central differences of the GPU loss itself.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from oracle import learned as Lr
from paper_1711_05519_amd import inputs as I
from paper_1711_05519_amd import rpca as R

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def setup_case(m, n, r, seed, dtype=torch.float64, alpha=0.1):
    x = I.gaussian_instance(m, n, r, alpha, 1.0, seed=seed)
    D = x.D if dtype == torch.float64 else x.D.astype(np.float32).astype(np.float64)
    p = O.Params(r=r, beta=x.beta, beta_init=x.beta_init, gamma=x.gamma, mu=x.mu_in, tol=1e-6)
    st = O.initialize(D, p)
    st = O.step(D, st, p)
    sv = R.Solver(dev(D, dtype), r, x.beta, x.beta_init, x.gamma, x.mu_in, training=True)
    sv.set_state(st.U, st.sigma, st.V, st.zeta, st.k, normD=O.frobenius(D))
    # ground truth as factors: L = P Q^T
    U, s, Vt = np.linalg.svd(x.L, full_matrices=False)
    P = U[:, :r] * s[:r]
    Q = Vt[:r].T
    return x, p, D, st, sv, P, Q


@pytest.mark.parametrize("m,n,r,seed", [(30, 30, 2, 5), (300, 250, 3, 11), (513, 700, 5, 12)])
def test_relaxed_step_fp64_matches_oracle(m, n, r, seed):
    say(f"relaxed step fp64 m={m} n={n} r={r}")
    x, p, D, st, sv, P, Q = setup_case(m, n, r, seed)
    saved = sv.get_state()
    for zs, ts in [(1.0, 0.05), (0.7, 0.2)]:
        sv.put_state(saved)
        zeta, tau = st.zeta * zs, st.zeta * ts
        res = sv.relaxed_step(zeta, tau, dev(P), dev(Q))
        L1, _, _, _ = Lr.relaxed_step(D, st, zeta, tau, p)
        loss_o = Lr.step_loss(D, st, zeta, tau, p, x.L)
        g_o = Lr.step_loss_grad_zeta(D, st, zeta, tau, p, x.L)
        U, s, V = (t.cpu().numpy() for t in sv.L_factors())
        assert rel((U * s) @ V.T, L1) < 1e-9
        assert res.loss == pytest.approx(loss_o, rel=1e-9)
        assert res.dloss_dzeta == pytest.approx(g_o, rel=1e-7, abs=1e-14 * abs(loss_o) / zeta)
        # relaxed err_k of the input state
        X = D - st.L()
        err_o = np.linalg.norm(X - Lr.soft_threshold(X, zeta, tau)) / np.linalg.norm(D)
        assert res.err == pytest.approx(err_o, rel=1e-10)
        assert sv.state.k == st.k + 1


def test_relaxed_step_derivative_against_gpu_differences():
    x, p, D, st, sv, P, Q = setup_case(400, 380, 4, 21)
    saved = sv.get_state()
    zeta, tau = st.zeta, 0.1 * st.zeta
    sv.put_state(saved)
    g = sv.relaxed_step(zeta, tau, dev(P), dev(Q)).dloss_dzeta

    def loss(z):
        sv.put_state(saved)
        return sv.relaxed_step(z, tau, dev(P), dev(Q)).loss

    # Fourth-order central difference. The loss is formed from reduced-space
    # inner products whose absolute rounding is ~1e-16, so the step must stay
    # well above that: h = 1e-3 zeta (truncation ~(h / tau)^4 = 1e-8 relative).
    h = 1e-3 * zeta
    fd = (8.0 * (loss(zeta + h) - loss(zeta - h)) - (loss(zeta + 2 * h) - loss(zeta - 2 * h))) / (12.0 * h)
    assert g == pytest.approx(fd, rel=1e-5)


def test_relaxed_step_fp32_data():
    x, p, D, st, sv, P, Q = setup_case(600, 500, 5, 31, dtype=torch.float32)
    zeta, tau = st.zeta, 0.05 * st.zeta
    res = sv.relaxed_step(zeta, tau, dev(P), dev(Q))
    loss_o = Lr.step_loss(D, st, zeta, tau, p, x.L)
    g_o = Lr.step_loss_grad_zeta(D, st, zeta, tau, p, x.L)
    assert res.loss == pytest.approx(loss_o, rel=1e-4)
    # FP32 bases and data: the derivative to 1e-3 of its natural scale loss / zeta
    assert abs(res.dloss_dzeta - g_o) <= 1e-3 * (abs(g_o) + loss_o / zeta)


def test_relaxed_step_autograd_function():
    x, p, D, st, sv, P, Q = setup_case(200, 210, 3, 41)
    zeta = torch.tensor(st.zeta, dtype=torch.float64, device="cuda", requires_grad=True)
    saved = sv.get_state()
    loss = R.RelaxedStep.apply(zeta, sv, dev(P), dev(Q), 0.1 * st.zeta)
    (g,) = torch.autograd.grad(2.0 * loss, zeta)
    sv.put_state(saved)
    ref = sv.relaxed_step(st.zeta, 0.1 * st.zeta, dev(P), dev(Q))
    assert float(g) == pytest.approx(2.0 * ref.dloss_dzeta, rel=1e-12)
    assert float(loss) == pytest.approx(ref.loss, rel=1e-12)


def test_relaxed_step_small_tau_is_the_hard_iteration():
    x, p, D, st, sv, P, Q = setup_case(300, 300, 3, 51)
    a = np.abs(D - st.L()).ravel()
    assert np.min(np.abs(a - st.zeta)) > 1e-6 * st.zeta
    sv.relaxed_step(st.zeta, 1e-10 * st.zeta, dev(P), dev(Q))
    nxt = O.step(D, st, p)
    U, s, V = (t.cpu().numpy() for t in sv.L_factors())
    assert rel((U * s) @ V.T, nxt.L()) < 1e-9
