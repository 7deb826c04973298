"""Seeded synthetic RPCA instances D = L + S.

This module only draws inputs. It holds none of the method's arithmetic: the
solver (GPU library) and the FP64 reference both receive the matrices built
here, so they solve bit-identical problems.

Recipes
-------
* Gaussian-factor instances (Section 3, "Synthetic Datasets"): L = P Q^T with
  P (m x r) and Q (n x r) drawn i.i.d. N(0, 1); the support of S is a set of
  round(alpha*m*n) positions drawn uniformly without replacement; the values of
  S are i.i.d. uniform on [-c*E|L_ij|, c*E|L_ij|], with E|L_ij| taken as the
  empirical mean of |L| over the generated matrix.
* Video-shaped instances (stand-in for the background-subtraction benchmark of
  Section 3, whose videos are not available here): pixels x frames with a
  rank-2 smooth background and moving 16x16 foreground blocks.

Draw order is fixed (P, Q, support, values) with numpy's PCG64 so a seed
reproduces an instance bit for bit.

Parameters follow the experiment section: the algorithm is given 1.1*mu where
mu is the incoherence of the true L, beta = 1.1*mu*r / (2*sqrt(m*n)),
beta_init = 1.1*mu*r / sqrt(m*n), gamma = 0.5 if alpha < 0.55 else 0.65.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 171105519


def seed_for(config: int, instance: int = 0) -> int:
    """Seed of instance `instance` of workload configuration `config`."""
    return SEED_BASE + 1000 * int(config) + int(instance)


@dataclasses.dataclass
class Instance:
    """One synthetic problem: D = L + S plus the parameters handed to the solver."""

    D: np.ndarray          # m x n float64, row-major
    L: np.ndarray | None   # ground-truth low-rank part (float64) or None if not kept
    P: np.ndarray          # left factor of L (m x r) - L = P Q^T
    Q: np.ndarray          # right factor of L (n x r)
    support: np.ndarray    # flat indices of the support of S (int64, sorted)
    r: int
    mu: float              # incoherence of the true L (assumption A1)
    mu_in: float           # value handed to the solver (1.1*mu)
    beta: float
    beta_init: float
    gamma: float
    tol: float
    alpha: float
    c: float
    seed: int

    @property
    def m(self) -> int:
        return self.D.shape[0]

    @property
    def n(self) -> int:
        return self.D.shape[1]


def incoherence(P: np.ndarray, Q: np.ndarray) -> float:
    """Incoherence mu of L = P Q^T in the sense of assumption A1.

    mu = max{ (m/r) max_i ||e_i^T U||^2 , (n/r) max_j ||e_j^T V||^2 } where U, V
    are orthonormal bases of the column and row spaces of L. Only the spans
    matter, so thin QR factors of P and Q are used.
    """
    m, r = P.shape
    n = Q.shape[0]
    Up, _ = np.linalg.qr(P)
    Vq, _ = np.linalg.qr(Q)
    mu_u = (m / r) * float(np.max(np.einsum("ij,ij->i", Up, Up)))
    mu_v = (n / r) * float(np.max(np.einsum("ij,ij->i", Vq, Vq)))
    return max(mu_u, mu_v)


def paper_parameters(m: int, n: int, r: int, mu: float, alpha: float,
                     gamma: float | None = None) -> dict:
    """Experiment-section parameter rule (1.1*mu, beta, beta_init, gamma)."""
    mu_in = 1.1 * mu
    beta = mu_in * r / (2.0 * math.sqrt(m * n))
    beta_init = mu_in * r / math.sqrt(m * n)
    if gamma is None:
        gamma = 0.5 if alpha < 0.55 else 0.65
    return dict(mu_in=mu_in, beta=beta, beta_init=beta_init, gamma=gamma)


def gaussian_instance(m: int, n: int, r: int, alpha: float, c: float, seed: int,
                      tol: float = 1e-5, keep_L: bool = True,
                      gamma: float | None = None) -> Instance:
    """Gaussian-factor instance of the synthetic-data experiments."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = rng.standard_normal((m, r))
    Q = rng.standard_normal((n, r))
    L = P @ Q.T
    k = int(round(alpha * m * n))
    support = np.sort(rng.choice(m * n, size=k, replace=False)).astype(np.int64)
    amp = c * float(np.mean(np.abs(L)))
    vals = rng.uniform(-amp, amp, size=k)
    D = L.copy()
    D.reshape(-1)[support] += vals
    mu = incoherence(P, Q)
    prm = paper_parameters(m, n, r, mu, alpha, gamma)
    return Instance(D=D, L=L if keep_L else None, P=P, Q=Q, support=support, r=r,
                    mu=mu, tol=tol, alpha=alpha, c=c, seed=seed, **prm)


# --- video-shaped instance -------------------------------------------------

VIDEO_H, VIDEO_W = 144, 176


def _smooth_field(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    """Sum of 8 random low-frequency 2-D cosines, min-max normalised to [0,1]."""
    y = np.arange(h)[:, None] / h
    x = np.arange(w)[None, :] / w
    f = np.zeros((h, w))
    for _ in range(8):
        kx, ky = rng.integers(0, 4, size=2)
        a = rng.standard_normal()
        ph = rng.uniform(0.0, 2.0 * math.pi)
        f += a * np.cos(math.pi * (kx * x + ky * y) + ph)
    f -= f.min()
    mx = f.max()
    return f / mx if mx > 0 else f


def _temporal_profile(rng: np.random.Generator, n: int, every: int = 100) -> np.ndarray:
    knots_t = np.arange(0, n + every, every)
    knots_v = rng.standard_normal(knots_t.size)
    return np.interp(np.arange(n), knots_t, knots_v)


def video_instance(n_frames: int = 2000, seed: int = 0, tol: float = 1e-5,
                   keep_L: bool = True, block: int = 16) -> Instance:
    """Video-shaped instance: (144*176) pixels x n_frames, rank-2 background.

    Column j is frame j vectorised row-major (pixel p = y*176 + x). S holds up
    to three moving block x block squares per frame with values U[-1, 1];
    track 0 is present in every frame, tracks 1 and 2 each on one contiguous
    interval of n_frames/4 frames; later tracks overwrite earlier ones.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    h, w = VIDEO_H, VIDEO_W
    m, n = h * w, n_frames
    F = np.stack([_smooth_field(rng, h, w).reshape(-1) for _ in range(2)], axis=1)
    T = np.stack([_temporal_profile(rng, n) for _ in range(2)], axis=1)
    L = F @ T.T
    frames = np.zeros((n, h, w))
    for trk in range(3):
        pos = np.array([rng.uniform(0, w - block), rng.uniform(0, h - block)])
        vel = rng.uniform(-1.5, 1.5, size=2)
        if trk == 0:
            t0, t1 = 0, n
        else:
            span = n // 4
            t0 = int(rng.integers(0, n - span + 1))
            t1 = t0 + span
        for t in range(n):
            if t0 <= t < t1:
                x0, y0 = int(pos[0]), int(pos[1])
                vals = rng.uniform(-1.0, 1.0, size=(block, block))
                frames[t, y0:y0 + block, x0:x0 + block] = vals
            pos += vel
            for d, lim in ((0, w - block), (1, h - block)):
                if pos[d] < 0:
                    pos[d] = -pos[d]
                    vel[d] = -vel[d]
                elif pos[d] > lim:
                    pos[d] = 2 * lim - pos[d]
                    vel[d] = -vel[d]
    S = np.ascontiguousarray(frames.reshape(n, m).T)
    del frames
    D = L + S
    support = np.flatnonzero(S.reshape(-1)).astype(np.int64)
    mu = incoherence(F, T)
    alpha = support.size / float(m * n)
    prm = paper_parameters(m, n, 2, mu, alpha, gamma=0.7)
    return Instance(D=D, L=L if keep_L else None, P=F, Q=T, support=support, r=2,
                    mu=mu, tol=tol, alpha=alpha, c=1.0, seed=seed, **prm)


# --- named workload configurations ------------------------------------------

def config_instance(config: int, instance: int = 0, keep_L: bool = True) -> Instance:
    """The five named workloads.

    1: 1000 x 1000, r=5, alpha=0.1, c=1, tol 1e-6 (FP64)
    2: 10000 x 10000, r=5, alpha=0.1, c=1, tol 1e-5
    3: video-shaped 25344 x 2000, r=2, gamma=0.7, tol 1e-5
    4: 20000 x 20000, r=10, alpha=0.2, c=1, tol 1e-5
    5: learned-threshold training pool: 2000 x 2000, r ~ U{5..10},
       alpha ~ U[0.05, 0.3], c ~ U[0.5, 2] (per instance)
    """
    s = seed_for(config, instance)
    if config == 1:
        return gaussian_instance(1000, 1000, 5, 0.1, 1.0, s, tol=1e-6, keep_L=keep_L, gamma=0.5)
    if config == 2:
        return gaussian_instance(10000, 10000, 5, 0.1, 1.0, s, tol=1e-5, keep_L=keep_L, gamma=0.5)
    if config == 3:
        return video_instance(2000, s, tol=1e-5, keep_L=keep_L)
    if config == 4:
        return gaussian_instance(20000, 20000, 10, 0.2, 1.0, s, tol=1e-5, keep_L=keep_L, gamma=0.5)
    if config == 5:
        rng = np.random.Generator(np.random.PCG64(s))
        r = int(rng.integers(5, 11))
        alpha = float(rng.uniform(0.05, 0.3))
        c = float(rng.uniform(0.5, 2.0))
        return gaussian_instance(2000, 2000, r, alpha, c, s + 500_000, tol=1e-5, keep_L=keep_L, gamma=0.5)
    raise ValueError(f"unknown configuration {config}")
