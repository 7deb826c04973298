"""Learned threshold schedule: the network's training kernels against the FP64
reference, and the loop's use of the network with its fallback.

Parity unpinned by the paper (it has no learned threshold). The network
kernels are FP32 and compared with the FP64 reference (itself pinned by finite
differences and closed forms in tests/test_oracle_learned.py) at 1e-5. The
fallback is pinned by construction: a network that returns NaN gives exactly
the paper's schedule; one that returns a huge threshold is abandoned after one
step that does not lower err_k, and the solve still converges.
"""
import math
import os
import sys

import numpy as np
import pytest
import torch

from oracle import learned as Lr
from paper_1711_05519_amd import inputs as I
from paper_1711_05519_amd import learn as LN
from paper_1711_05519_amd import rpca as R

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def f32dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


def test_mlp_forward_backward_adam_against_reference():
    rng = np.random.default_rng(7)
    th = (Lr.init_theta(2) + 0.2 * rng.standard_normal(Lr.N_PARAMS)).astype(np.float32).astype(np.float64)
    B = 37
    phi = rng.standard_normal((B, 4)).astype(np.float32).astype(np.float64)
    go = rng.standard_normal(B).astype(np.float32).astype(np.float64)
    o = R.rpca_mlp_forward(f32dev(th), f32dev(phi)).cpu().numpy()
    ref = np.array([Lr.mlp_forward(th, phi[b])[0] for b in range(B)])
    assert np.allclose(o, ref, rtol=1e-5, atol=1e-5)
    g = R.rpca_mlp_backward(f32dev(th), f32dev(phi), f32dev(go)).cpu().numpy()
    gref = sum(Lr.mlp_backward(th, Lr.mlp_forward(th, phi[b])[1], go[b]) for b in range(B))
    assert np.abs(g - gref).max() <= 1e-5 * max(1.0, np.abs(gref).max())
    # two Adam steps
    t_th, t_m, t_v = f32dev(th), torch.zeros(Lr.N_PARAMS, device="cuda"), torch.zeros(Lr.N_PARAMS, device="cuda")
    rth, rm, rv = th.copy(), np.zeros(Lr.N_PARAMS), np.zeros(Lr.N_PARAMS)
    for t in (1, 2):
        R.rpca_mlp_adam(t_th, t_m, t_v, f32dev(gref * t), t, 1e-3)
        rth, rm, rv = Lr.adam_step(rth, rm, rv, (gref * t).astype(np.float32).astype(np.float64), t, 1e-3)
    assert np.abs(t_th.cpu().numpy() - rth).max() < 1e-6


def test_features_agree_with_reference():
    a = LN.features(3, 100.0, 1.0, 1e-2, 1e4)
    b = Lr.features(3, 15, 100.0, 1.0, 1e-2, 1e4)
    assert np.allclose(a, b, rtol=1e-15)


def _solve(x, theta, D32):
    sv = R.Solver(D32, x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol, seed=7, learned=theta)
    info = sv.solve()
    U, s, V = (t.cpu().numpy() for t in sv.L_factors())
    return info, (U * s) @ V.T


def test_learned_nan_network_falls_back_to_the_paper_schedule():
    x = I.config_instance(1, keep_L=True)
    D32 = torch.as_tensor(x.D, dtype=torch.float32, device="cuda")
    th = LN.init_theta(0)
    th[-1] = float("nan")
    ip, Lp = _solve(x, None, D32)
    il, Ll = _solve(x, th, D32)
    assert ip.iterations == il.iterations
    assert np.array_equal(np.asarray(ip.err_hist), np.asarray(il.err_hist))
    assert np.array_equal(Lp, Ll)


def test_learned_huge_threshold_is_abandoned_and_the_solve_converges():
    x = I.config_instance(1, keep_L=True)
    D32 = torch.as_tensor(x.D, dtype=torch.float32, device="cuda")
    th = LN.init_theta(0)
    th[-1] = 60.0          # clipped to exp(5): zeta ~ 150 times the paper's
    il, Ll = _solve(x, th, D32)
    assert il.status == R.RPCA_OK and il.err < x.tol
    assert np.linalg.norm(Ll - x.L) / np.linalg.norm(x.L) <= 1e-4


def test_learned_untrained_network_is_the_paper_schedule():
    x = I.config_instance(1, keep_L=True)
    D32 = torch.as_tensor(x.D, dtype=torch.float32, device="cuda")
    ip, Lp = _solve(x, None, D32)
    il, Ll = _solve(x, LN.init_theta(0), D32)   # o = 0 exactly: exp(0) = 1
    assert il.status == R.RPCA_OK
    assert np.array_equal(np.asarray(ip.err_hist), np.asarray(il.err_hist))


def test_shipped_network_converges_on_held_out_instances():
    path = os.path.join(os.path.dirname(LN.__file__), "zeta_mlp.npy")
    if not os.path.exists(path):
        pytest.skip("no trained network shipped")
    th = LN.load_theta(path)
    for i in (512, 513):
        x = I.config_instance(5, i, keep_L=True)
        D32 = torch.as_tensor(x.D, dtype=torch.float32, device="cuda")
        ip, _ = _solve(x, None, D32)
        il, Ll = _solve(x, th, D32)
        say(f"held-out {i}: r={x.r} alpha={x.alpha:.3f} plain {ip.iterations} it, learned {il.iterations} it")
        assert il.status == R.RPCA_OK
        assert np.linalg.norm(Ll - x.L) / np.linalg.norm(x.L) <= 1e-4
