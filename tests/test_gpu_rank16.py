"""Whole solves at the largest rank the loop supports (r = 16): FP64 against
the FP64 oracle (same iteration count, L within 1e-10), FP32 and the mixed
form (BF16 products) against the truth. At this rank the streaming passes'
workgroup 0 completes each loop update's sums of Grams and cross products
(Cholesky factors of 16 x 16 Grams) in the FP32, FP64 and BF16 passes alike."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1711_05519_amd import inputs as I
from paper_1711_05519_amd import rpca as R

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_factored(U, s, V, L):
    return float(np.linalg.norm((U * s) @ V.T - L) / np.linalg.norm(L))


@pytest.mark.parametrize("form", ["fp64", "fp32", "mixed"])
def test_solve_at_rank_16(form):
    m, n, r = 600, 520, 16
    fp64 = form == "fp64"
    x = I.gaussian_instance(m, n, r, 0.05, 1.0, seed=16, tol=1e-7 if fp64 else 1e-5)
    dtype = torch.float64 if fp64 else torch.float32
    D = torch.as_tensor(x.D, dtype=dtype, device="cuda")
    sv = R.Solver(D, r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol, seed=1, mixed=form == "mixed")
    info = sv.solve()
    U, s, V = (t.cpu().numpy() for t in sv.L_factors())
    L_true = x.P @ x.Q.T
    rec = rel_factored(U, s, V, L_true)
    say(f"r = 16, {form}: {info.iterations} iterations, err {info.err:.2e}, recovery {rec:.2e}")
    assert info.status == R.RPCA_OK and info.err < x.tol
    assert rec <= 1e-4
    if fp64:
        p = O.Params(r=r, beta=x.beta, beta_init=x.beta_init, gamma=x.gamma, mu=x.mu_in, tol=x.tol)
        ref = O.solve(x.D, p)
        d = rel_factored(U, s, V, ref.state.L())
        say(f"  oracle: {ref.iterations} iterations, rel L to the oracle {d:.2e}")
        assert info.iterations == ref.iterations
        assert d <= 1e-10
