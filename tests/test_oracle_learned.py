"""Pins of the FP64 reference for the learned-threshold extension (CPU only).

The paper has no learned threshold, so these references are pinned by
mathematics instead: central finite differences of every derivative, closed
forms (an Adam step at t = 1, the untrained output), and limits (the relaxed
threshold tends to T_zeta as tau -> 0, the relaxed iteration to Algorithm 1).
"""
import numpy as np
import pytest

import oracle as O
from oracle import learned as Lr
from paper_1711_05519_amd import inputs as I


def test_mlp_layout_and_untrained_output():
    assert Lr.N_PARAMS == 1249
    th = Lr.init_theta(0)
    # the untrained network outputs o = 0 exactly: the paper's threshold
    o, _ = Lr.mlp_forward(th, np.array([0.3, -2.0, -1.0, -4.0]))
    assert o == 0.0
    assert Lr.zeta_of(o, 7.5) == 7.5
    # zero first-layer weights give o = b3 exactly, and the correction is clipped
    z = th.copy()
    z[:Lr.N_H * Lr.N_IN] = 0.0
    z[-1] = 0.7
    assert Lr.mlp_forward(z, np.array([1.0, 2.0, 3.0, 4.0]))[0] == pytest.approx(0.7, abs=1e-15)
    assert Lr.zeta_of(40.0, 2.0) == pytest.approx(2.0 * np.exp(5.0), rel=1e-15)


def test_mlp_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    th = Lr.init_theta(3) + 0.2 * rng.standard_normal(Lr.N_PARAMS)
    phi = np.array([0.2, -1.5, -2.5, -3.0])
    o, cache = Lr.mlp_forward(th, phi)
    g = Lr.mlp_backward(th, cache, 1.0)
    h = 1e-6
    for i in rng.choice(Lr.N_PARAMS, 60, replace=False).tolist() + [Lr.N_PARAMS - 1]:
        e = np.zeros_like(th)
        e[i] = h
        fd = (Lr.mlp_forward(th + e, phi)[0] - Lr.mlp_forward(th - e, phi)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, abs=1e-7, rel=1e-6), i


def test_adam_first_step_closed_form():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    th1, m, v = Lr.adam_step(th, np.zeros(3), np.zeros(3), g, 1, lr=0.1, eps=1e-8)
    # at t = 1 the bias-corrected moments are g and g^2
    assert np.allclose(th1, th - 0.1 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features():
    f = Lr.features(3, 15, sigma1=100.0, sigma_r1=1.0, err=1e-2, normD=1e4)
    assert np.allclose(f, [0.2, np.log(0.01), np.log(1e-2), np.log(0.01)])
    assert np.isfinite(Lr.features(0, 15, 1.0, 0.0, 0.0, 1.0)).all()
    # sigma_{r+1} / sigma_1 is clamped at 1e-4 (unresolved below in FP32)
    assert Lr.features(1, 15, 1.0, 1e-9, 1e-3, 1.0)[1] == pytest.approx(np.log(1e-4))
    assert Lr.features(1, 15, 2.0, 0.0, 1e-3, 1.0)[1] == pytest.approx(np.log(1e-4))
    assert Lr.features(1, 15, 2.0, 4e-4, 1e-3, 1.0)[1] == pytest.approx(np.log(2e-4))


def test_soft_threshold_limit_and_derivative():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(2000) * 3
    zeta = 2.0
    far = np.abs(np.abs(x) - zeta) > 0.05
    s = Lr.soft_threshold(x, zeta, 1e-4)
    assert np.array_equal(s[far], O.hard_threshold(x, zeta)[far])
    tau, h = 0.3, 1e-6
    fd = (Lr.soft_threshold(x, zeta + h, tau) - Lr.soft_threshold(x, zeta - h, tau)) / (2 * h)
    assert np.allclose(Lr.soft_threshold_dzeta(x, zeta, tau), fd, rtol=1e-6, atol=1e-8)


def test_truncation_derivative_matches_central_differences():
    rng = np.random.default_rng(4)
    m, n, r = 12, 9, 3
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.array([9.0, 7.0, 5.0, 2.0, 1.5, 1.0, 0.7, 0.4, 0.1])
    Amat = (U[:, :n] * s) @ V.T
    E = rng.standard_normal((m, n))
    h = 1e-6

    def Hr(X):
        a, b, c = O.best_rank_r(X, r)
        return (a * b) @ c.T
    fd = (Hr(Amat + h * E) - Hr(Amat - h * E)) / (2 * h)
    an = Lr.truncation_derivative(Amat, E, r)
    assert np.abs(an - fd).max() < 1e-7 * np.abs(fd).max()


def _tiny_case(seed=5):
    x = I.gaussian_instance(30, 30, 2, 0.1, 1.0, seed=seed)
    p = O.Params(r=2, beta=x.beta, beta_init=x.beta_init, gamma=x.gamma, mu=x.mu_in, tol=1e-6)
    D = x.D
    st = O.initialize(D, p)
    st = O.step(D, st, p)
    return x, p, D, st


def test_step_loss_grad_zeta_matches_central_differences():
    x, p, D, st = _tiny_case()
    L_true = x.L
    for zeta_scale, tau_scale in [(1.0, 0.05), (0.6, 0.2), (1.5, 0.02)]:
        zeta = st.zeta * zeta_scale
        tau = zeta * tau_scale
        g = Lr.step_loss_grad_zeta(D, st, zeta, tau, p, L_true)
        h = 1e-6 * zeta
        fd = (Lr.step_loss(D, st, zeta + h, tau, p, L_true) - Lr.step_loss(D, st, zeta - h, tau, p, L_true)) / (2 * h)
        assert g == pytest.approx(fd, rel=2e-5, abs=1e-12), (zeta_scale, tau_scale, g, fd)


def test_relaxed_step_tends_to_algorithm_1():
    x, p, D, st = _tiny_case(6)
    nxt = O.step(D, st, p)
    # zeta strictly between entries of |D - L_k|: the relaxation with a tiny tau
    # reproduces the hard-threshold iteration
    L1, _, _, _ = Lr.relaxed_step(D, st, st.zeta, 1e-9 * st.zeta, p)
    a = np.abs(D - st.L()).ravel()
    assert np.min(np.abs(a - st.zeta)) > 1e-6 * st.zeta
    assert np.abs(L1 - nxt.L()).max() < 1e-9 * np.abs(nxt.L()).max()


# ------------------------------------------- Algorithm 1 with the network ---

def _small_case(seed=77, r=3, tol=1e-9):
    x = I.gaussian_instance(120, 100, r, 0.1, 1.0, seed=seed, tol=tol)
    p = O.Params(r=r, beta=x.beta, beta_init=x.beta_init, gamma=x.gamma, mu=x.mu_in, tol=tol)
    return x, p


def _bias_only(b3):
    th = np.zeros(Lr.N_PARAMS)
    th[-1] = b3
    return th


def test_learned_solve_without_network_is_algorithm_1():
    x, p = _small_case()
    ref = O.solve(x.D, p)
    for th in (None, Lr.init_theta(4)):          # no network, and the untrained one (o = 0 exactly)
        got = Lr.learned_solve(x.D, p, th)
        assert got.iterations == ref.iterations
        assert got.err_hist == ref.err_hist and got.zeta_hist == ref.zeta_hist
        assert np.array_equal(got.state.L(), ref.state.L())
    assert Lr.learned_solve(x.D, p, None).learned_hist == [False] * ref.iterations
    assert Lr.learned_solve(x.D, p, Lr.init_theta(4)).learned_hist[0]


def test_learned_solve_nan_network_falls_back_at_once():
    x, p = _small_case()
    th = _bias_only(np.nan)
    got = Lr.learned_solve(x.D, p, th)
    ref = O.solve(x.D, p)
    assert not any(got.learned_hist)
    assert got.err_hist == ref.err_hist and np.array_equal(got.state.L(), ref.state.L())


def test_learned_solve_bias_network_scales_the_threshold_step_by_step():
    # o = b3 = -2 for every input: each learned threshold is e^-2 times the
    # paper's (low enough that S_k grows and err_k falls from the first body,
    # so the latch stays open). Composed from independent bodies of
    # Algorithm 1 whose threshold is replaced by the scaled one.
    x, p = _small_case()
    D = x.D
    f = np.exp(-2.0)
    got = Lr.learned_solve(D, p, _bias_only(-2.0), fixed_iters=3)
    nD = O.frobenius(D)
    st = O.initialize(D, p, nD)
    assert got.zeta_hist[0] == st.zeta and got.err_hist[0] == st.err
    for k in range(3):
        nxt = O.step(D, st, p, nD)                           # the paper's body from the same state
        paper = O.next_zeta(p.beta, p.gamma, k, nxt.sigma_M, p.r)
        assert got.learned_hist[k]
        assert got.zeta_hist[k + 1] == pytest.approx(f * paper, rel=1e-14)
        np.testing.assert_allclose(got.sigma_hist[k], nxt.sigma_M, rtol=1e-12)
        st = O.State(U=nxt.U, sigma=nxt.sigma, V=nxt.V, zeta=f * paper, k=k + 1)
        L1 = st.L()
        st.err = O.relative_error(D, L1, O.hard_threshold(D - L1, st.zeta), nD)
        assert got.err_hist[k + 1] == pytest.approx(st.err, rel=1e-10)
        assert got.err_hist[k + 1] < got.err_hist[k]      # so the latch stays open
    assert np.linalg.norm(got.state.L() - st.L()) <= 1e-10 * np.linalg.norm(st.L())


def test_learned_solve_plateau_closes_the_latch():
    # While the thresholds exceed every corrupted entry, S_k stays empty and
    # err_k does not fall (err_1 = err_0 up to rounding on this instance): a
    # network that keeps the thresholds that high is used for zeta_1 only.
    x, p = _small_case()
    got = Lr.learned_solve(x.D, p, _bias_only(np.log(2.0)))
    assert got.err_hist[1] >= got.err_hist[0]
    assert got.learned_hist[0] and not any(got.learned_hist[1:])
    assert got.converged


def test_learned_solve_latch_returns_to_the_paper_schedule():
    # A threshold e^5 times the paper's absorbs too little into S: err rises,
    # and from that iterate on every threshold is Algorithm 1's again, and the
    # solve still reaches the tolerance.
    x, p = _small_case()
    got = Lr.learned_solve(x.D, p, _bias_only(60.0))
    first_rise = next(k for k in range(1, len(got.err_hist)) if got.err_hist[k] >= got.err_hist[k - 1])
    assert got.learned_hist[:first_rise] == [True] * first_rise
    assert not any(got.learned_hist[first_rise:])
    for k in range(first_rise, got.iterations):
        assert got.zeta_hist[k + 1] == O.next_zeta(p.beta, p.gamma, k, got.sigma_hist[k], p.r)
    for k in range(first_rise):
        paper = O.next_zeta(p.beta, p.gamma, k, got.sigma_hist[k], p.r)
        assert got.zeta_hist[k + 1] == pytest.approx(np.exp(5.0) * paper, rel=1e-14)
    assert got.converged
    assert O.recovery_error(got.state.L(), x.L) <= 1e-4
