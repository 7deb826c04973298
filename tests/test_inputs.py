"""Seeded generators: reproducibility and the recipe of Section 3."""
import math

import numpy as np

from paper_1711_05519_amd import inputs as I


def test_seed_reproduces_bit_for_bit():
    a = I.gaussian_instance(200, 150, 3, 0.1, 1.0, seed=5)
    b = I.gaussian_instance(200, 150, 3, 0.1, 1.0, seed=5)
    c = I.gaussian_instance(200, 150, 3, 0.1, 1.0, seed=6)
    assert np.array_equal(a.D, b.D) and np.array_equal(a.support, b.support)
    assert not np.array_equal(a.D, c.D)


def test_gaussian_recipe():
    x = I.gaussian_instance(300, 200, 4, 0.2, 2.0, seed=9)
    assert x.support.size == round(0.2 * 300 * 200)
    assert np.unique(x.support).size == x.support.size
    assert np.linalg.matrix_rank(x.L) == 4
    S = x.D - x.L
    amp = 2.0 * np.mean(np.abs(x.L))
    vals = S.reshape(-1)[x.support]
    assert np.all(np.abs(vals) <= amp) and np.abs(vals).max() > 0.9 * amp
    off = np.ones(S.size, bool)
    off[x.support] = False
    assert not S.reshape(-1)[off].any()
    # parameter rule of the experiment section
    assert math.isclose(x.mu_in, 1.1 * x.mu)
    assert math.isclose(x.beta, 1.1 * x.mu * 4 / (2 * math.sqrt(300 * 200)))
    assert math.isclose(x.beta_init, 2 * x.beta)
    assert x.gamma == 0.5
    assert I.gaussian_instance(50, 50, 2, 0.6, 1.0, seed=1).gamma == 0.65


def test_incoherence_definition():
    rng = np.random.default_rng(0)
    P = rng.standard_normal((80, 3))
    Q = rng.standard_normal((60, 3))
    U, s, Vt = np.linalg.svd(P @ Q.T, full_matrices=False)
    mu = max(80 / 3 * (U[:, :3] ** 2).sum(1).max(), 60 / 3 * (Vt[:3].T ** 2).sum(1).max())
    assert math.isclose(I.incoherence(P, Q), mu, rel_tol=1e-10)
    assert 1.0 <= mu <= 60 / 3


def test_video_recipe():
    x = I.video_instance(n_frames=160, seed=3)
    assert x.m == 144 * 176 and x.n == 160 and x.r == 2
    assert np.linalg.matrix_rank(x.L, tol=1e-8 * np.abs(x.L).max()) == 2
    S = x.D - x.L
    per_frame = (S != 0).sum(0) / 256.0
    assert per_frame.min() >= 0.5 and per_frame.max() <= 3.0
    assert 0.005 < x.alpha < 0.03
    assert np.abs(S).max() <= 1.0
    assert x.gamma == 0.7


def test_config_seeds_distinct():
    assert len({I.seed_for(c, i) for c in range(1, 6) for i in range(600)}) == 5 * 600
