"""FP64 CPU references for the learned-threshold extension (test infrastructure).

Not part of the paper: the paper fixes the threshold schedule
zeta_{k+1} = beta (sigma_{r+1} + gamma^{k+1} sigma_1) (Algorithm 1, Section 2.1).
This module is the plain reference for the additions built on top of it:

* a small multilayer perceptron that maps features of the current iterate to a
  correction of the threshold, zeta_k = zeta_paper * exp(clip(o, -5, 5))
  (4 -> 32 -> 32 -> 1, ReLU hidden layers), its gradient and one Adam update
  (Kingma and Ba, "Adam: a method for stochastic optimization", Algorithm 1);
* one AccAltProj iteration with the hard threshold T_zeta replaced by the
  relaxation s(x) = x * logistic((|x| - zeta) / tau), which tends to T_zeta as
  tau -> 0, together with the derivative of a loss of the next iterate with
  respect to zeta;
* Algorithm 1 whose thresholds come from the network, with the fallback to
  the paper's schedule once err_k stops decreasing (learned_solve).

Everything is dense float64 and literal: the derivative of the rank-r
truncation H_r is the first-order perturbation of a full dense SVD, written
out below. Parity of these functions is not pinned by the paper (it has no
learned threshold); the tests pin them by central finite differences, closed
forms and limits instead.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import accaltproj as A

# ---------------------------------------------------------------- the MLP ----

N_IN, N_H = 4, 32
# flat parameter layout: W1 (32x4, row-major), b1 (32), W2 (32x32), b2 (32), w3 (32), b3 (1)
SIZES = (N_H * N_IN, N_H, N_H * N_H, N_H, N_H, 1)
N_PARAMS = sum(SIZES)          # 1249
FEATURE_FLOOR = 1e-30          # floor inside the logarithms of the features
# sigma_{r+1} / sigma_1 is clamped from below: a library that computes the
# singular values of M in FP32 products resolves sigma_{r+1} only to about
# 1e-5 sigma_1, so smaller ratios would feed rounding noise to the network
SIGMA_RATIO_FLOOR = 1e-4


def unpack(theta: np.ndarray):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, o = [], 0
    for sz in SIZES:
        out.append(theta[o:o + sz])
        o += sz
    W1, b1, W2, b2, w3, b3 = out
    return W1.reshape(N_H, N_IN), b1, W2.reshape(N_H, N_H), b2, w3, b3[0]


def features(k: int, K: int, sigma1: float, sigma_r1: float, err: float, normD: float) -> np.ndarray:
    """phi_k = (k / K, log max(sigma_{r+1} / sigma_1, 1e-4), log err_k, log(sigma_1 / ||D||_F))."""
    f = FEATURE_FLOOR
    return np.array([k / K,
                     np.log(max(sigma_r1 / max(sigma1, f), SIGMA_RATIO_FLOOR)),
                     np.log(max(err, f)),
                     np.log(max(sigma1, f) / max(normD, f))], dtype=np.float64)


def mlp_forward(theta: np.ndarray, phi: np.ndarray):
    """Returns (o, cache): o = w3 . relu(W2 relu(W1 phi + b1) + b2) + b3."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    a1 = W1 @ phi + b1
    h1 = np.maximum(a1, 0.0)
    a2 = W2 @ h1 + b2
    h2 = np.maximum(a2, 0.0)
    o = float(w3 @ h2 + b3)
    return o, (phi, a1, h1, a2, h2)


O_CLIP = 5.0


def zeta_of(o: float, zeta_paper: float) -> float:
    """zeta = zeta_paper * exp(clip(o, -5, 5)); zeta_paper the schedule of Algorithm 1."""
    return zeta_paper * float(np.exp(np.clip(o, -O_CLIP, O_CLIP)))


def mlp_backward(theta: np.ndarray, cache, grad_o: float) -> np.ndarray:
    """d(grad_o * o)/d theta, flat, by the chain rule through the two ReLU layers."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    phi, a1, h1, a2, h2 = cache
    g_w3 = grad_o * h2
    g_b3 = grad_o
    g_h2 = grad_o * w3
    g_a2 = g_h2 * (a2 > 0)
    g_W2 = np.outer(g_a2, h1)
    g_b2 = g_a2
    g_h1 = W2.T @ g_a2
    g_a1 = g_h1 * (a1 > 0)
    g_W1 = np.outer(g_a1, phi)
    g_b1 = g_a1
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])


def adam_step(theta, m, v, g, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_theta(seed: int) -> np.ndarray:
    """He-style normal weights, zero biases and a zero output layer: the
    untrained output is o = 0, i.e. the paper's schedule."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((N_H, N_IN)) * np.sqrt(2.0 / N_IN)
    W2 = rng.standard_normal((N_H, N_H)) * np.sqrt(2.0 / N_H)
    return np.concatenate([W1.ravel(), np.zeros(N_H), W2.ravel(), np.zeros(N_H), np.zeros(N_H), [0.0]])


# ------------------------------------------------ relaxed iteration ---------

def logistic(u):
    return 0.5 * (1.0 + np.tanh(0.5 * u))


def soft_threshold(x: np.ndarray, zeta: float, tau: float) -> np.ndarray:
    """s(x) = x * logistic((|x| - zeta) / tau); T_zeta(x) in the limit tau -> 0."""
    return x * logistic((np.abs(x) - zeta) / tau)


def soft_threshold_dzeta(x: np.ndarray, zeta: float, tau: float) -> np.ndarray:
    """d s / d zeta = -x * logistic'(u) / tau, u = (|x| - zeta) / tau."""
    g = logistic((np.abs(x) - zeta) / tau)
    return -x * g * (1.0 - g) / tau


def relaxed_step(D: np.ndarray, st: A.State, zeta: float, tau: float, p: A.Params):
    """One iteration of Algorithm 1 from L_k = st.L() with the relaxed threshold:
    Z = D - s(D - L_k); L_{k+1} = H_r(P_T(Z)) with T from Trim(L_k).
    Returns (L_{k+1}, P_T(Z), Ut, Vt)."""
    Ut, Vt = A.trimmed_bases(st.U, st.V, p.mu, p.r)
    X = D - st.L()
    Z = D - soft_threshold(X, zeta, tau)
    PZ = A.tangent_projection(Ut, Vt, Z)
    U, s, V = A.best_rank_r(PZ, p.r)
    return (U * s) @ V.T, PZ, Ut, Vt


def step_loss(D, st, zeta, tau, p, L_true) -> float:
    """||L_{k+1} - L_true||_F^2 / ||L_true||_F^2 after one relaxed iteration."""
    L1, _, _, _ = relaxed_step(D, st, zeta, tau, p)
    return float(np.sum((L1 - L_true) ** 2) / np.sum(L_true ** 2))


def truncation_derivative(Amat: np.ndarray, E: np.ndarray, r: int) -> np.ndarray:
    """First-order change of H_r(Amat) in the direction E, from the full SVD
    Amat = U diag(s) V^T: with F = U^T E V, the change is U G V^T where
    G_ij = F_ij for i, j < r; for i < r <= j (s_j = 0 past min(m, n)),
    G_ij = (s_i^2 F_ij + s_i s_j F_ji) / (s_i^2 - s_j^2) and
    G_ji = (s_i^2 F_ji + s_i s_j F_ij) / (s_i^2 - s_j^2); G_ij = 0 for i, j >= r.
    (Requires s_{r-1} > s_r.)"""
    m, n = Amat.shape
    U, s, Vt = np.linalg.svd(Amat, full_matrices=True)
    V = Vt.T
    sf = np.zeros(max(m, n))
    sf[:len(s)] = s
    F = U.T @ E @ V
    G = np.zeros_like(F)
    G[:r, :r] = F[:r, :r]
    for i in range(r):
        for j in range(r, n):
            G[i, j] = (sf[i] ** 2 * F[i, j] + sf[i] * sf[j] * (F[j, i] if j < m else 0.0)) / (sf[i] ** 2 - sf[j] ** 2)
        for j in range(r, m):
            G[j, i] = (sf[i] ** 2 * F[j, i] + sf[i] * sf[j] * (F[i, j] if j < n else 0.0)) / (sf[i] ** 2 - sf[j] ** 2)
    return U @ G @ V.T


def step_loss_grad_zeta(D, st, zeta, tau, p, L_true) -> float:
    """d step_loss / d zeta: Z depends on zeta through s, P_T is linear, and
    H_r changes by truncation_derivative in the direction P_T(dZ/dzeta)."""
    L1, PZ, Ut, Vt = relaxed_step(D, st, zeta, tau, p)
    X = D - st.L()
    dZ = -soft_threshold_dzeta(X, zeta, tau)
    dPZ = A.tangent_projection(Ut, Vt, dZ)
    dL1 = truncation_derivative(PZ, dPZ, p.r)
    return float(2.0 * np.sum((L1 - L_true) * dL1) / np.sum(L_true ** 2))


# ------------------------------------------- Algorithm 1 with the network ---

K_FEAT = 15          # iteration count that normalises the first feature


@dataclasses.dataclass
class LearnedSolve:
    state: A.State
    err_hist: list
    zeta_hist: list
    sigma_hist: list     # sigma_M of P_T(D - S_k) for every executed body (k = 0, 1, ...)
    learned_hist: list   # whether zeta_{k+1} came from the network
    iterations: int
    converged: bool


def learned_solve(D: np.ndarray, p: A.Params, theta: np.ndarray | None, max_iter: int | None = None,
                  fixed_iters: int | None = None) -> LearnedSolve:
    """Algorithm 1 (with the initialisation of Algorithm 3) in which the
    threshold of every body may come from the network:

      zeta_{k+1} = zeta_paper * exp(clip(o_k, -5, 5)),
      zeta_paper = beta (sigma_{r+1} + gamma^{k+1} sigma_1)   (Algorithm 1),
      o_k = network(phi_k),  phi_k = ((k + 1) / 15, log max(sigma_{r+1} / sigma_1, 1e-4),
                                      log err_k, log(sigma_1 / ||D||_F)),

    with sigma_1, sigma_{r+1} those of P_T(D - S_k) (the 2r x 2r matrix of
    Section 2.1). Fallback latch: once err_k >= err_{k-1} (k >= 1), or once the
    network's threshold is not a positive finite number, every later threshold
    is the paper's. theta None means the paper's schedule throughout. The
    stopping rule is Section 3's (err_k < tol or k = max_iter); fixed_iters
    runs exactly that many bodies instead. theta is used as given (the network
    of the library holds FP32 parameters: pass them rounded to FP32)."""
    if max_iter is None:
        max_iter = p.max_iter
    normD = A.frobenius(D)
    st = A.initialize(D, p, normD)
    err_hist, zeta_hist, sigma_hist, learned_hist = [st.err], [st.zeta], [], []
    on = theta is not None
    err_prev = math.inf
    while True:
        k = st.k
        if on and k >= 1 and not (st.err < err_prev):
            on = False                       # err stopped decreasing: the paper's schedule from here on
        err_prev = st.err
        if fixed_iters is not None:
            if k >= fixed_iters:
                break
        elif st.err < p.tol or k >= max_iter:
            break
        # one body of Algorithm 1: Trim, H_r(P_T(D - S_k)), then the threshold
        Sk = A.hard_threshold(D - st.L(), st.zeta)
        Ut, Vt = A.trimmed_bases(st.U, st.V, p.mu, p.r)
        ts = A.tangent_svd(Ut, Vt, D - Sk, p.r)
        zeta = A.next_zeta(p.beta, p.gamma, k, ts.sigma_M, p.r)
        used = False
        if on:
            phi = features(k + 1, K_FEAT, float(ts.sigma_M[0]), float(ts.sigma_M[p.r]), st.err, normD)
            o, _ = mlp_forward(theta, phi)
            zl = zeta_of(o, zeta) if o == o else math.nan
            if math.isfinite(zl) and zl > 0.0:
                zeta, used = zl, True
            else:
                on = False
        nxt = A.State(U=ts.U, sigma=ts.sigma, V=ts.V, zeta=zeta, k=k + 1, sigma_M=ts.sigma_M)
        L1 = nxt.L()
        nxt.err = A.relative_error(D, L1, A.hard_threshold(D - L1, zeta), normD)
        st = nxt
        err_hist.append(st.err)
        zeta_hist.append(st.zeta)
        sigma_hist.append(ts.sigma_M.copy())
        learned_hist.append(used)
    return LearnedSolve(state=st, err_hist=err_hist, zeta_hist=zeta_hist, sigma_hist=sigma_hist,
                        learned_hist=learned_hist, iterations=st.k, converged=bool(st.err < p.tol))
