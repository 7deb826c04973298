"""Plain FP64 AccAltProj on the CPU - the correctness oracle (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module. It is deliberately slow and literal: every matrix is dense float64 and
every step is written in the order and notation of the paper
(Cai, Cai, Wei - "Accelerated Alternating Projections for Robust Principal
Component Analysis"):

* Algorithm 1 (AccAltProj loop), Algorithm 2 (Trim), Algorithm 3
  (initialisation by two steps of modified AltProj);
* Section 2.1: the tangent space T_k, its projection P_T, the complement
  projection, H_r, the fast SVD of P_T(D - S_k) through a 2r x 2r matrix M_k,
  the hard-thresholding operator T_zeta and the threshold schedule zeta_k;
* Section 3: the relative error err_k and the stopping rule.

Library primitives (matrix products, Householder QR, dense LAPACK SVD and the
ARPACK truncated SVD for large matrices) serve as single steps; nothing is
blocked, fused or reordered.

Readings taken where the paper is silent or garbled (each is listed with its
reason in the design notes of the repository):
* Trim levels: rows of U use sqrt(mu*r/m), rows of V use sqrt(mu*r/n)
  (assumption A1); a zero row keeps weight 1; the Trim output is
  L~ = A Sigma B^T and only orthonormal bases of span(A), span(B) are used.
* The second complement is (I - V~V~^T)(D - S_k)^T U~ (transpose of D - S_k).
* T_zeta keeps entries with |x| > zeta strictly.
* sigma_{r+1}(P_T(D - S_k)) is the (r+1)-th singular value of M_k (0-based
  index r); the first loop threshold uses gamma^1.
* The stopping test err_k < tol is applied at the top of each iteration.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse.linalg as spla

# Dense LAPACK SVD up to this many entries; ARPACK truncated SVD above.
DENSE_SVD_MAX_ENTRIES = 4_000_000


# --------------------------------------------------------------------------
# Elementary operators
# --------------------------------------------------------------------------

def frobenius(X: np.ndarray) -> float:
    """||X||_F (notation paragraph of Section 1.2)."""
    return float(np.linalg.norm(X))


def hard_threshold(Z: np.ndarray, zeta: float) -> np.ndarray:
    """T_zeta (Section 2.1): keep Z_ij where |Z_ij| > zeta, zero elsewhere."""
    return np.where(np.abs(Z) > zeta, Z, 0.0)


def relative_error(D: np.ndarray, L: np.ndarray, S: np.ndarray, normD: float | None = None) -> float:
    """err_k = ||D - L_k - S_k||_F / ||D||_F (Section 3, relative computing error)."""
    if normD is None:
        normD = frobenius(D)
    return frobenius(D - L - S) / normD


def _sorted_truncated_svd(Z: np.ndarray, k: int):
    """Top-k singular triplets of Z in descending order.

    Dense LAPACK SVD for small matrices; for large ones ARPACK (svds) run to
    machine precision (tol=0) from a fixed start, as the paper does with a
    Lanczos-type truncated SVD for large D (Section 3).
    """
    m, n = Z.shape
    if m * n <= DENSE_SVD_MAX_ENTRIES or k >= min(m, n) - 1:
        U, s, Vt = np.linalg.svd(Z, full_matrices=False)
        return U[:, :k], s[:k], Vt[:k, :].T
    v0 = np.ones(min(m, n)) / math.sqrt(min(m, n))
    U, s, Vt = spla.svds(Z, k=k, tol=0, v0=v0, solver="arpack")
    order = np.argsort(s)[::-1]
    return U[:, order], s[order], Vt[order, :].T


def best_rank_r(Z: np.ndarray, r: int):
    """H_r (Section 2.1, eq. for H_r): best rank-r approximation by SVD truncation.

    Returns (U, sigma, V) with H_r(Z) = U diag(sigma) V^T.
    """
    return _sorted_truncated_svd(Z, r)


def sigma_1(Z: np.ndarray) -> float:
    """Largest singular value sigma_1(Z)."""
    _, s, _ = _sorted_truncated_svd(Z, 1)
    return float(s[0])


# --------------------------------------------------------------------------
# Algorithm 2 - Trim
# --------------------------------------------------------------------------

def trim(U: np.ndarray, V: np.ndarray, mu: float, r: int):
    """Algorithm 2: scale row i of U by min{1, c/||U^(i)||} (same for V).

    Returns the trimmed factors (A, B); the trimmed matrix is A Sigma B^T.
    """
    m, n = U.shape[0], V.shape[0]
    c_u = math.sqrt(mu * r / m)
    c_v = math.sqrt(mu * r / n)

    def scale_rows(X, c):
        out = np.empty_like(X)
        for i in range(X.shape[0]):
            rho = float(np.linalg.norm(X[i]))
            w = 1.0 if rho == 0.0 else min(1.0, c / rho)
            out[i] = w * X[i]
        return out

    return scale_rows(U, c_u), scale_rows(V, c_v)


def orthonormal_basis(A: np.ndarray) -> np.ndarray:
    """Orthonormal basis of span(A) by Householder QR (footnote to Section 2.1)."""
    Q, _ = np.linalg.qr(A)
    return Q


def trimmed_bases(U: np.ndarray, V: np.ndarray, mu: float, r: int):
    """U~_k, V~_k: orthonormal bases of the trimmed factors (Trim + QR).

    mu <= 0 selects AccAltProj without trim (Section 3): U~ = U, V~ = V.
    """
    if mu <= 0:
        return U.copy(), V.copy()
    A, B = trim(U, V, mu, r)
    return orthonormal_basis(A), orthonormal_basis(B)


# --------------------------------------------------------------------------
# Section 2.1 - tangent space projection and the fast H_r(P_T(.))
# --------------------------------------------------------------------------

def tangent_projection(Ut: np.ndarray, Vt: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """P_T Z = U U^T Z + Z V V^T - U U^T Z V V^T (Section 2.1), dense."""
    UUt = Ut @ Ut.T
    VVt = Vt @ Vt.T
    return UUt @ Z + Z @ VVt - UUt @ Z @ VVt


def tangent_complement(Ut: np.ndarray, Vt: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """(I - P_T) Z = (I - U U^T) Z (I - V V^T) (Section 2.1), dense."""
    m, n = Z.shape
    return (np.eye(m) - Ut @ Ut.T) @ Z @ (np.eye(n) - Vt @ Vt.T)


@dataclasses.dataclass
class TangentSVD:
    """Everything the fast H_r(P_T Z) produces (Section 2.1)."""

    U: np.ndarray        # [U~ Q1] U_M[:, :r]
    sigma: np.ndarray    # Sigma_M[:r]
    V: np.ndarray        # [V~ Q2] V_M[:, :r]
    sigma_M: np.ndarray  # all 2r singular values of M (= those of P_T Z)
    Y1: np.ndarray       # Z V~
    Y2: np.ndarray       # Z^T U~
    C: np.ndarray        # U~^T Z V~
    Q1: np.ndarray
    R1: np.ndarray
    Q2: np.ndarray
    R2: np.ndarray
    M: np.ndarray


def tangent_svd(Ut: np.ndarray, Vt: np.ndarray, Z: np.ndarray, r: int, keep: int | None = None) -> TangentSVD:
    """Fast SVD of P_T Z through the 2r x 2r matrix M (Section 2.1).

    (I - U~U~^T) Z V~ = Q1 R1 and (I - V~V~^T) Z^T U~ = Q2 R2 (thin QR);
    M = [[U~^T Z V~, R2^T], [R1, 0]];  M = U_M Sigma_M V_M^T;
    new factors [U~ Q1] U_M, Sigma_M, [V~ Q2] V_M truncated to the top `keep`
    (default r) triplets, which is H_r(P_T Z).
    """
    if keep is None:
        keep = r
    Y1 = Z @ Vt
    Y2 = Z.T @ Ut
    C = Ut.T @ Y1
    W1 = Y1 - Ut @ C
    W2 = Y2 - Vt @ (Vt.T @ Y2)
    Q1, R1 = np.linalg.qr(W1)
    Q2, R2 = np.linalg.qr(W2)
    k = Ut.shape[1]
    M = np.zeros((2 * k, 2 * k))
    M[:k, :k] = C
    M[:k, k:] = R2.T
    M[k:, :k] = R1
    UM, sM, VMt = np.linalg.svd(M)
    Unew = np.hstack([Ut, Q1]) @ UM[:, :keep]
    Vnew = np.hstack([Vt, Q2]) @ VMt.T[:, :keep]
    return TangentSVD(U=Unew, sigma=sM[:keep].copy(), V=Vnew, sigma_M=sM, Y1=Y1, Y2=Y2,
                      C=C, Q1=Q1, R1=R1, Q2=Q2, R2=R2, M=M)


def next_zeta(beta: float, gamma: float, k: int, sigma_M: np.ndarray, r: int) -> float:
    """zeta_{k+1} = beta (sigma_{r+1}(P_T Z) + gamma^{k+1} sigma_1(P_T Z)) (Algorithm 1)."""
    return beta * (float(sigma_M[r]) + gamma ** (k + 1) * float(sigma_M[0]))


# --------------------------------------------------------------------------
# Iterate state and Algorithms 1 and 3
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Params:
    r: int
    beta: float
    beta_init: float
    gamma: float
    mu: float            # trim level handed to Trim; <= 0 disables trimming
    tol: float = 1e-5
    max_iter: int = 100  # Section 3: at most 100 iterations


@dataclasses.dataclass
class State:
    """(L_k, S_k) with L_k = U diag(sigma) V^T and S_k = T_zeta(D - L_k)."""

    U: np.ndarray
    sigma: np.ndarray
    V: np.ndarray
    zeta: float
    k: int
    err: float = float("nan")
    sigma_M: np.ndarray | None = None  # singular values of P_T(D - S_{k-1}) that produced this state

    def L(self) -> np.ndarray:
        return (self.U * self.sigma) @ self.V.T

    def S(self, D: np.ndarray) -> np.ndarray:
        return hard_threshold(D - self.L(), self.zeta)


@dataclasses.dataclass
class InitTrace:
    sigma1_D: float
    zeta_m1: float       # zeta_{-1}
    S_m1: np.ndarray     # S_{-1}
    sigma1_Z: float      # sigma_1(D - S_{-1})


def initialize(D: np.ndarray, p: Params, normD: float | None = None, trace: bool = False):
    """Algorithm 3: initialisation by two steps of modified AltProj.

    L_{-1} = 0; zeta_{-1} = beta_init sigma_1(D); S_{-1} = T(D - L_{-1});
    L_0 = H_r(D - S_{-1}); zeta_0 = beta sigma_1(D - S_{-1});
    S_0 = T_{zeta_0}(D - L_0).
    """
    if normD is None:
        normD = frobenius(D)
    s1D = sigma_1(D)
    zeta_m1 = p.beta_init * s1D
    L_m1 = np.zeros_like(D)
    S_m1 = hard_threshold(D - L_m1, zeta_m1)
    U0, s0, V0 = best_rank_r(D - S_m1, p.r)
    zeta0 = p.beta * float(s0[0])       # sigma_1(D - S_{-1}) is the top singular value
    st = State(U=U0, sigma=s0, V=V0, zeta=zeta0, k=0)
    L0 = st.L()
    S0 = hard_threshold(D - L0, zeta0)
    st.err = relative_error(D, L0, S0, normD)
    if trace:
        return st, InitTrace(sigma1_D=s1D, zeta_m1=zeta_m1, S_m1=S_m1, sigma1_Z=float(s0[0]))
    return st


def step(D: np.ndarray, st: State, p: Params, normD: float | None = None) -> State:
    """One pass of the body of Algorithm 1, from (L_k, S_k) to (L_{k+1}, S_{k+1})."""
    if normD is None:
        normD = frobenius(D)
    k = st.k
    Lk = st.L()
    Sk = hard_threshold(D - Lk, st.zeta)
    Ut, Vt = trimmed_bases(st.U, st.V, p.mu, p.r)          # L~_k = Trim(L_k, mu)
    ts = tangent_svd(Ut, Vt, D - Sk, p.r)                  # L_{k+1} = H_r(P_T~(D - S_k))
    zeta = next_zeta(p.beta, p.gamma, k, ts.sigma_M, p.r)  # zeta_{k+1}
    nxt = State(U=ts.U, sigma=ts.sigma, V=ts.V, zeta=zeta, k=k + 1, sigma_M=ts.sigma_M)
    Lk1 = nxt.L()
    Sk1 = hard_threshold(D - Lk1, zeta)                    # S_{k+1} = T(D - L_{k+1})
    nxt.err = relative_error(D, Lk1, Sk1, normD)
    return nxt


@dataclasses.dataclass
class SolveResult:
    state: State
    err_hist: list
    zeta_hist: list
    iterations: int
    converged: bool


def solve(D: np.ndarray, p: Params, max_iter: int | None = None, fixed_iters: int | None = None) -> SolveResult:
    """Algorithm 1 with the initialisation of Algorithm 3.

    Loop while err_k >= tol and k < max_iter (Section 3: stop when err_k < tol
    or after 100 iterations). With `fixed_iters` the loop runs exactly that many
    bodies regardless of err_k (used to compare trajectories step for step).
    """
    if max_iter is None:
        max_iter = p.max_iter
    normD = frobenius(D)
    st = initialize(D, p, normD)
    err_hist = [st.err]
    zeta_hist = [st.zeta]
    while True:
        if fixed_iters is not None:
            if st.k >= fixed_iters:
                break
        elif st.err < p.tol or st.k >= max_iter:
            break
        st = step(D, st, p, normD)
        err_hist.append(st.err)
        zeta_hist.append(st.zeta)
    return SolveResult(state=st, err_hist=err_hist, zeta_hist=zeta_hist, iterations=st.k,
                       converged=bool(st.err < p.tol))


def recovery_error(L_est: np.ndarray, L_true: np.ndarray) -> float:
    """||L_k - L||_F / ||L||_F, the success criterion of Section 3 (<= 1e-4)."""
    return frobenius(L_est - L_true) / frobenius(L_true)
