"""Pins of the FP64 reference adjoint of unrolled relaxed bodies
(oracle/adjoint.py) by central finite differences of its own forward, an
adjoint identity of the truncation derivative, and the one-body threshold
derivative of the learned-threshold module."""
import math

import numpy as np
import pytest

from oracle import accaltproj as A
from oracle import adjoint as J
from oracle import learned as Lr


def instance(m=26, n=22, r=2, alpha=0.1, seed=3, mu=1.2):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((m, r))
    Q = rng.standard_normal((n, r))
    T = P @ Q.T
    S = np.zeros((m, n))
    sup = rng.random((m, n)) < alpha
    S[sup] = rng.uniform(-1.0, 1.0, sup.sum()) * 2.0 * np.mean(np.abs(T))
    D = T + S
    U0, s0, V0 = A.best_rank_r(T + 0.3 * rng.standard_normal((m, n)), r)
    p = A.Params(r=r, beta=0.5, beta_init=1.0, gamma=0.6, mu=mu)
    zetas = [0.9 * np.max(np.abs(T)) * 0.6 ** k for k in range(4)]
    return D, P, Q, U0, s0, V0, p, zetas


def fd(f, h=1e-6):
    return (f(h) - f(-h)) / (2 * h)


def test_truncation_adjoint_identity():
    rng = np.random.default_rng(1)
    for (m, n, rank, r) in [(9, 7, 4, 2), (7, 9, 4, 2), (8, 8, 8, 3)]:
        Y = rng.standard_normal((m, rank)) @ rng.standard_normal((rank, n))
        E = rng.standard_normal((m, n))
        G = rng.standard_normal((m, n))
        lhs = float(np.sum(Lr.truncation_derivative(Y, E, r) * G))
        rhs = float(np.sum(E * J.truncation_adjoint(Y, G, r)))
        assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + 1.0), (m, n, lhs, rhs)


def test_soft_derivatives():
    x = np.linspace(-3, 3, 41)
    for zeta, tau in [(1.0, 0.2), (0.5, 0.05)]:
        d1 = fd(lambda h: J.soft(x + h, zeta, tau))
        d2 = fd(lambda h: J.soft(x, zeta + h, tau))
        assert np.allclose(J.soft_dx(x, zeta, tau), d1, rtol=1e-6, atol=1e-7)
        assert np.allclose(J.soft_dzeta(x, zeta, tau), d2, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("mu", [1.2, 0.0])
def test_one_body_gradients_match_central_differences(mu):
    D, P, Q, U0, s0, V0, p, zetas = instance(mu=mu)
    if mu > 0:
        cU, cV = J.trim_levels(*D.shape, p.mu, p.r)
        assert np.any(np.linalg.norm(U0, axis=1) > cU) and np.any(np.linalg.norm(V0, axis=1) > cV)
    z, t = zetas[:1], [0.2 * zetas[0]]
    w = [1.0]
    adj = J.unrolled_adjoint(D, U0, s0, V0, z, t, w, p, P, Q)
    rng = np.random.default_rng(11)
    dU, ds, dV = rng.standard_normal(U0.shape), rng.standard_normal(s0.shape), rng.standard_normal(V0.shape)
    f = lambda h: J.unrolled_loss(D, U0 + h * dU, s0 + h * ds, V0 + h * dV, z, t, w, p, P, Q)
    an = float(np.sum(adj.Ubar0 * dU) + adj.sbar0 @ ds + np.sum(adj.Vbar0 * dV))
    assert abs(fd(f) - an) <= 1e-6 * abs(an), (fd(f), an)
    g = lambda h: J.unrolled_loss(D, U0, s0, V0, [z[0] + h], t, w, p, P, Q)
    assert abs(fd(g) - adj.zeta_bar[0]) <= 1e-6 * abs(adj.zeta_bar[0])
    # the one-body threshold derivative of the learned-threshold module
    st = A.State(U=U0, sigma=s0, V=V0, zeta=z[0], k=0)
    ref = Lr.step_loss_grad_zeta(D, st, z[0], t[0], p, P @ Q.T)
    assert abs(ref - adj.zeta_bar[0]) <= 1e-9 * abs(ref)
    assert abs(adj.loss - Lr.step_loss(D, st, z[0], t[0], p, P @ Q.T)) <= 1e-12


def test_unrolled_gradients_match_central_differences():
    D, P, Q, U0, s0, V0, p, zetas = instance()
    K = 4
    t = [0.2 * z for z in zetas]
    w = [0.25, 0.0, 0.5, 1.0]
    adj = J.unrolled_adjoint(D, U0, s0, V0, zetas, t, w, p, P, Q)
    assert adj.loss == pytest.approx(J.unrolled_loss(D, U0, s0, V0, zetas, t, w, p, P, Q), rel=1e-13)
    for k in range(K):
        def g(h, k=k):
            zz = list(zetas)
            zz[k] += h
            return J.unrolled_loss(D, U0, s0, V0, zz, t, w, p, P, Q)
        num = fd(g)
        assert abs(num - adj.zeta_bar[k]) <= 1e-5 * max(abs(num), 1e-3 * np.max(np.abs(adj.zeta_bar))), (k, num)
    rng = np.random.default_rng(12)
    dU, ds, dV = rng.standard_normal(U0.shape), rng.standard_normal(s0.shape), rng.standard_normal(V0.shape)
    f = lambda h: J.unrolled_loss(D, U0 + h * dU, s0 + h * ds, V0 + h * dV, zetas, t, w, p, P, Q)
    an = float(np.sum(adj.Ubar0 * dU) + adj.sbar0 @ ds + np.sum(adj.Vbar0 * dV))
    assert abs(fd(f) - an) <= 1e-5 * abs(an), (fd(f), an)


def test_chained_gradient_is_the_gradient_in_L():
    """Between bodies the gradient is taken with respect to L_k: along a
    tangent direction of the rank-r matrices at L_1 (moved by H_r), the
    two-body loss changes by <Lbar_1, E>."""
    D, P, Q, U0, s0, V0, p, zetas = instance(seed=5)
    t = [0.2 * z for z in zetas[:2]]
    b0 = J.relaxed_body(D, U0, s0, V0, zetas[0], t[0], p)
    U1, s1, V1 = b0.U1, b0.s1, b0.V1
    nt = float(np.sum((P @ Q.T) ** 2))
    b1 = J.relaxed_body(D, U1, s1, V1, zetas[1], t[1], p)
    L2 = (b1.U1 * b1.s1) @ b1.V1.T
    adj = J.body_adjoint(D, b1, p, 2.0 * (L2 - P @ Q.T) / nt)
    rng = np.random.default_rng(2)
    E = U1 @ rng.standard_normal((p.r, D.shape[1])) + rng.standard_normal((D.shape[0], p.r)) @ V1.T

    def f(h):
        Uh, sh, Vh = A.best_rank_r((U1 * s1) @ V1.T + h * E, p.r)
        return J.unrolled_loss(D, Uh, sh, Vh, zetas[1:2], t[1:2], [1.0], p, P, Q)

    an = float(np.sum(adj.Lbar * E))
    assert abs(fd(f) - an) <= 1e-5 * abs(an), (fd(f), an)
