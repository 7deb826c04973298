"""FP64 CPU reference of the reverse-mode adjoint of unrolled relaxed AccAltProj
iterations (test infrastructure; only the tests use it).

Not part of the paper. It differentiates K bodies of Algorithm 1 in which the
hard threshold T_zeta is replaced by the relaxation
s(x) = x * logistic((|x| - zeta) / tau) (T_zeta as tau -> 0), for a training
loss of the iterates sum_k w_k ||L_k - P Q^T||_F^2 / ||P Q^T||_F^2 (P Q^T the
known low-rank part of a synthetic instance). One body, from free factors
(U, sigma, V) of L_k = U diag(sigma) V^T:

  Trim (Algorithm 2):  A = diag(w_U) U, w_U,i = min(1, c_U / ||U_i||), c_U = sqrt(mu r / m);
                       B = diag(w_V) V likewise; U~, V~ orthonormal bases of span(A), span(B)
  X = D - L_k,  Z = D - s(X)
  Y = P_T(Z) = U~U~^T Z + Z V~V~^T - U~U~^T Z V~V~^T      (Section 2.1)
  L_{k+1} = H_r(Y),  factors (U', sigma', V') from its SVD

Everything here is dense and literal; the derivatives are written out from the
chain rule in the order of that body, reversed:

* H_r: from the full SVD Y = U_Y diag(s) V_Y^T, the change of H_r(Y) in a
  direction E is U_Y Phi(U_Y^T E V_Y) V_Y^T with Phi the coefficient map of
  the first-order perturbation of the top-r singular triplets (requires
  s_{r-1} > s_r); the adjoint applies the transpose of Phi;
* P_T: linear in Z (its adjoint is itself), and bilinear in the projectors
  P_U = U~U~^T, P_V = V~V~^T: dY = dP_U Z (I - P_V) + (I - P_U) Z dP_V;
* orthonormal basis of span(A): P_U = A (A^T A)^{-1} A^T, whose differential
  is (I - P_U) dA A^+ + (A^+)^T dA^T (I - P_U);
* Trim: the row weights w_i = c / ||U_i|| where ||U_i|| > c (constant 1 where
  not);
* the relaxation: dZ/dL = s'(X) elementwise, dZ/dzeta = X g (1 - g) / tau with
  g = logistic((|X| - zeta) / tau), s'(x) = g + |x| g (1 - g) / tau.

Between bodies the loss depends on the state only through L_k (Trim uses the
row norms and the span of the orthonormal factor U_k, both functions of L_k),
so the gradient handed from body k to body k-1 is the dense dL_k; at the first
body the gradients with respect to the free factors (U_0, sigma_0, V_0) are
returned. The thresholds zeta_k are inputs (a learned schedule's features are
treated as constants).

Parity of these functions is not pinned by the paper; the tests pin them by
central finite differences of the forward below, an adjoint identity for Phi,
and the one-body derivative of the learned-threshold module.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import accaltproj as A


def logistic(u):
    return 0.5 * (1.0 + np.tanh(0.5 * u))


def soft(x, zeta, tau):
    """s(x) = x * logistic((|x| - zeta) / tau)."""
    return x * logistic((np.abs(x) - zeta) / tau)


def soft_dx(x, zeta, tau):
    """s'(x) = g + |x| g (1 - g) / tau."""
    g = logistic((np.abs(x) - zeta) / tau)
    return g + np.abs(x) * g * (1.0 - g) / tau


def soft_dzeta(x, zeta, tau):
    """ds/dzeta = -x g (1 - g) / tau."""
    g = logistic((np.abs(x) - zeta) / tau)
    return -x * g * (1.0 - g) / tau


def trim_levels(m: int, n: int, mu: float, r: int):
    """c_U = sqrt(mu r / m), c_V = sqrt(mu r / n) (Algorithm 2); None without trim."""
    if mu <= 0:
        return None, None
    return math.sqrt(mu * r / m), math.sqrt(mu * r / n)


def trim_rows(X: np.ndarray, c):
    """Row weights of Algorithm 2 and the row norms: w_i = min(1, c / ||X_i||), 1 for a zero row."""
    rho = np.linalg.norm(X, axis=1)
    if c is None:
        return np.ones(X.shape[0]), rho
    w = np.ones(X.shape[0])
    big = rho > c
    w[big] = c / rho[big]
    return w, rho


@dataclasses.dataclass
class Body:
    """The dense intermediates of one relaxed body."""

    U: np.ndarray
    sigma: np.ndarray
    V: np.ndarray
    zeta: float
    tau: float
    wU: np.ndarray
    rhoU: np.ndarray
    wV: np.ndarray
    rhoV: np.ndarray
    Am: np.ndarray       # A = diag(w_U) U
    Bm: np.ndarray       # B = diag(w_V) V
    Ut: np.ndarray       # U~
    Vt: np.ndarray       # V~
    X: np.ndarray
    Z: np.ndarray
    Y: np.ndarray        # P_T(Z)
    U1: np.ndarray       # factors of L_{k+1} = H_r(Y)
    s1: np.ndarray
    V1: np.ndarray


def relaxed_body(D: np.ndarray, U, sigma, V, zeta: float, tau: float, p: A.Params) -> Body:
    """One relaxed body of Algorithm 1 from free factors (U, sigma, V)."""
    m, n = D.shape
    cU, cV = trim_levels(m, n, p.mu, p.r)
    wU, rhoU = trim_rows(U, cU)
    wV, rhoV = trim_rows(V, cV)
    Am = wU[:, None] * U
    Bm = wV[:, None] * V
    Ut = A.orthonormal_basis(Am)
    Vt = A.orthonormal_basis(Bm)
    X = D - (U * sigma) @ V.T
    Z = D - soft(X, zeta, tau)
    Y = A.tangent_projection(Ut, Vt, Z)
    U1, s1, V1 = A.best_rank_r(Y, p.r)
    return Body(U=U, sigma=np.asarray(sigma, dtype=np.float64), V=V, zeta=zeta, tau=tau, wU=wU, rhoU=rhoU,
                wV=wV, rhoV=rhoV, Am=Am, Bm=Bm, Ut=Ut, Vt=Vt, X=X, Z=Z, Y=Y, U1=U1, s1=s1, V1=V1)


def unrolled_forward(D, U0, s0, V0, zetas, taus, p: A.Params):
    """K relaxed bodies from (U0, s0, V0) with thresholds zetas[k], temperatures taus[k]."""
    bodies = []
    U, s, V = U0, np.asarray(s0, dtype=np.float64), V0
    for z, t in zip(zetas, taus):
        b = relaxed_body(D, U, s, V, float(z), float(t), p)
        bodies.append(b)
        U, s, V = b.U1, b.s1, b.V1
    return bodies


def unrolled_loss(D, U0, s0, V0, zetas, taus, weights, p: A.Params, P, Q) -> float:
    """sum_{k=1..K} w_k ||L_k - P Q^T||_F^2 / ||P Q^T||_F^2."""
    bodies = unrolled_forward(D, U0, s0, V0, zetas, taus, p)
    T = P @ Q.T
    nt = float(np.sum(T * T))
    return float(sum(w * np.sum(((b.U1 * b.s1) @ b.V1.T - T) ** 2) / nt for w, b in zip(weights, bodies)))


# ---------------------------------------------------------------- adjoints ----

def truncation_adjoint(Y: np.ndarray, G: np.ndarray, r: int) -> np.ndarray:
    """Adjoint of the first-order change of H_r at Y: returns Ybar with
    <dH_r(Y)[E], G> = <E, Ybar> for every E. From the full SVD of Y, the change
    is U_Y Phi(U_Y^T E V_Y) V_Y^T with Phi(F)_ij = F_ij (i, j < r), and for
    i < r <= j: Phi_ij = (s_i^2 F_ij + s_i s_j F_ji) / (s_i^2 - s_j^2),
    Phi_ji = (s_i^2 F_ji + s_i s_j F_ij) / (s_i^2 - s_j^2) (s_j = 0 past
    min(m, n), and a missing partner entry counts as 0); the adjoint gathers,
    for every entry of F, the coefficients with which it enters Phi."""
    m, n = Y.shape
    U, s, Vt = np.linalg.svd(Y, full_matrices=True)
    V = Vt.T
    sf = np.zeros(max(m, n))
    sf[:len(s)] = s
    Gc = U.T @ G @ V                 # coordinates of G: Gc_ab = <u_a v_b^T, G>
    Fb = np.zeros_like(Gc)           # Fb_ab = sum over Phi entries of d Phi / d F_ab * Gc
    Fb[:r, :r] = Gc[:r, :r]
    for i in range(r):
        for j in range(r, max(m, n)):
            den = sf[i] ** 2 - sf[j] ** 2
            a = sf[i] ** 2 / den
            b = sf[i] * sf[j] / den
            gij = Gc[i, j] if j < n else 0.0     # Phi_ij exists when j < n
            gji = Gc[j, i] if j < m else 0.0     # Phi_ji exists when j < m
            if j < n:                             # F_ij enters Phi_ij (a) and Phi_ji (b)
                Fb[i, j] += a * gij + b * gji
            if j < m:                             # F_ji enters Phi_ji (a) and Phi_ij (b)
                Fb[j, i] += a * gji + b * gij
    return U @ Fb @ V.T


@dataclasses.dataclass
class BodyAdjoint:
    zeta_bar: float
    Lbar: np.ndarray      # gradient with respect to L_k (the loss as a function of L_k)
    Ubar: np.ndarray      # gradients with respect to the free factors of L_k
    sbar: np.ndarray
    Vbar: np.ndarray


def body_adjoint(D, b: Body, p: A.Params, Lbar1: np.ndarray) -> BodyAdjoint:
    """Reverse mode of one relaxed body: Lbar1 = dloss/dL_{k+1} (dense)."""
    m, n = D.shape
    cU, cV = trim_levels(m, n, p.mu, p.r)
    # L_{k+1} = H_r(Y)
    Ybar = truncation_adjoint(b.Y, Lbar1, p.r)
    # Y = P_T(Z): linear in Z, bilinear in the projectors
    PU = b.Ut @ b.Ut.T
    PV = b.Vt @ b.Vt.T
    Zbar = A.tangent_projection(b.Ut, b.Vt, Ybar)
    PUbar = Ybar @ (np.eye(n) - PV) @ b.Z.T
    PVbar = b.Z.T @ (np.eye(m) - PU) @ Ybar
    # P_U = A (A^T A)^{-1} A^T
    Abar = (np.eye(m) - PU) @ (PUbar + PUbar.T) @ b.Am @ np.linalg.inv(b.Am.T @ b.Am)
    Bbar = (np.eye(n) - PV) @ (PVbar + PVbar.T) @ b.Bm @ np.linalg.inv(b.Bm.T @ b.Bm)

    # Trim: A_i = w_i U_i, w_i = c / ||U_i|| where ||U_i|| > c
    def trim_adjoint(Xf, w, rho, c, Xbar_t):
        out = w[:, None] * Xbar_t
        if c is not None:
            for i in range(Xf.shape[0]):
                if rho[i] > c:
                    out[i] -= (c / rho[i] ** 3) * float(Xbar_t[i] @ Xf[i]) * Xf[i]
        return out

    Utrim = trim_adjoint(b.U, b.wU, b.rhoU, cU, Abar)
    Vtrim = trim_adjoint(b.V, b.wV, b.rhoV, cV, Bbar)
    # Z = D - s(D - L_k)
    LZ = Zbar * soft_dx(b.X, b.zeta, b.tau)
    zeta_bar = float(np.sum(Zbar * (-soft_dzeta(b.X, b.zeta, b.tau))))
    S = np.diag(b.sigma)
    Ubar = LZ @ b.V @ S + Utrim
    Vbar = LZ.T @ b.U @ S + Vtrim
    sbar = np.einsum("it,ij,jt->t", b.U, LZ, b.V)
    # as a function of L_k (orthonormal U, V): Trim sees the projectors only
    Si = np.diag(1.0 / b.sigma)
    Lbar = (LZ + (np.eye(m) - b.U @ b.U.T) @ Utrim @ Si @ b.V.T
            + b.U @ Si @ ((np.eye(n) - b.V @ b.V.T) @ Vtrim).T)
    return BodyAdjoint(zeta_bar=zeta_bar, Lbar=Lbar, Ubar=Ubar, sbar=sbar, Vbar=Vbar)


@dataclasses.dataclass
class UnrolledAdjoint:
    loss: float
    losses: list          # the K terms ||L_k - P Q^T||^2 / ||P Q^T||^2 (unweighted)
    zeta_bar: np.ndarray  # dloss / dzeta_k, k = 0..K-1
    Ubar0: np.ndarray     # dloss / d(U_0, sigma_0, V_0) as free factors
    sbar0: np.ndarray
    Vbar0: np.ndarray


def unrolled_adjoint(D, U0, s0, V0, zetas, taus, weights, p: A.Params, P, Q) -> UnrolledAdjoint:
    """Loss of K relaxed bodies and its gradients with respect to every
    threshold and to the initial factors (reverse sweep over the bodies)."""
    bodies = unrolled_forward(D, U0, s0, V0, zetas, taus, p)
    T = P @ Q.T
    nt = float(np.sum(T * T))
    K = len(bodies)
    losses = []
    for b in bodies:
        R = (b.U1 * b.s1) @ b.V1.T - T
        losses.append(float(np.sum(R * R) / nt))
    loss = float(sum(w * l for w, l in zip(weights, losses)))
    zbar = np.zeros(K)
    Lbar = np.zeros_like(D)
    adj = None
    for k in range(K - 1, -1, -1):
        b = bodies[k]
        Lbar = Lbar + 2.0 * weights[k] * ((b.U1 * b.s1) @ b.V1.T - T) / nt   # the term of L_{k+1}
        adj = body_adjoint(D, b, p, Lbar)
        zbar[k] = adj.zeta_bar
        Lbar = adj.Lbar
    return UnrolledAdjoint(loss=loss, losses=losses, zeta_bar=zbar, Ubar0=adj.Ubar, sbar0=adj.sbar, Vbar0=adj.Vbar)
