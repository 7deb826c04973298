"""Mixed-precision form (RPCA_FLAG_MIXED): of the tangent products
Y1 = Z V_f = L V_f + E V_f and Y2 = Z^T U_f = L^T U_f + E^T U_f (Z = D - S,
E = D - L - S), the residual parts E V_f and E^T U_f run on the matrix cores
with BF16 operands and FP32 accumulation and the rank-r parts are added
exactly from the factors; the threshold and the residual in FP32, small
algebra in FP64, as in the FP32 path.

Parity unpinned by the paper (a precision choice of this implementation).
Pins used instead: Y1 and Y2 against FP64 references computed from the
BF16-rounded operands (the kernel's own rounding, so agreement up to FP32
accumulation is required); the errors of Y1 and Y2 against the exact
products, which must scale with the size of E rather than with that of Z; the
threshold residual against the FP64 oracle at the FP32 tolerance; and whole
solves against the FP64 oracle and the ground truth at the 1e-4 level of the
paper's success criterion (Section 4).
"""
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


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def bf16(a):
    """Round-to-nearest-even to BF16 (as v_cvt_pk_bf16_f32 does), back in FP64."""
    t = torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64)
    return t.numpy()


@pytest.mark.parametrize("m,n,r", [(300, 270, 3), (64, 520, 1), (1031, 259, 5), (200, 200, 16), (97, 1000, 7),
                                   (517, 300, 10), (1000, 257, 8)])
def test_mixed_tangent_products(m, n, r):
    say(f"mixed tangent_products m={m} n={n} r={r}")
    rng = np.random.default_rng(10 * m + n + r)
    D = f32(rng.standard_normal((m, n)) * 2.0)
    A = f32(rng.standard_normal((m, r)))
    B = f32(rng.standard_normal((n, r)) / np.sqrt(r))
    Ut = f32(np.linalg.qr(rng.standard_normal((m, r)))[0])
    Vt = f32(np.linalg.qr(rng.standard_normal((n, r)))[0])
    x = D - A @ B.T
    a = np.sort(np.abs(x).reshape(-1))
    zeta = 0.5 * (a[int(0.8 * a.size)] + a[int(0.8 * a.size) + 1])
    S = np.where(np.abs(x) > zeta, x, 0.0)
    Z = D - S
    E = np.where(np.abs(x) <= zeta, x, 0.0)
    res_o = float(np.sum(E * E))
    # the operands of the matrix-core products: E, V_t and U_t rounded to BF16;
    # the rank-r parts L V_t = A (B^T V_t) and L^T U_t = B (A^T U_t) are exact
    Eb, Vb, Ub = bf16(E), bf16(Vt), bf16(Ut)
    Y1b = Eb @ Vb + A @ (B.T @ Vt)
    Y2b = Eb.T @ Ub + B @ (A.T @ Ut)
    Y1o, Y2o = Z @ Vt, Z.T @ Ut
    sv = R.Solver(dev(D, torch.float32), r, 0.01, 0.02, 0.5, 1.0, mixed=True)
    Y1, Y2, res = sv.tangent_products(dev(A), dev(B), zeta, dev(Ut), dev(Vt))
    Y1, Y2 = Y1.cpu().numpy(), Y2.cpu().numpy()
    # FP32 rebuild of L can move a value of E across a BF16 rounding boundary:
    # a few one-ulp differences of the operands, hence 1e-4 rather than FP32 eps
    assert rel(Y1, Y1b) < 1e-4, rel(Y1, Y1b)
    assert rel(Y2, Y2b) < 1e-4, rel(Y2, Y2b)
    # and the BF16 products are the exact products to BF16 accuracy
    assert rel(Y1, Y1o) < 2e-2
    assert rel(Y2, Y2o) < 2e-2
    # the residual is the FP32 path's
    assert abs(res - res_o) / res_o < 2e-6


@pytest.mark.parametrize("noise", [1e-2, 1e-4])
def test_mixed_error_scales_with_residual(noise):
    """Near convergence D - L is small: the BF16 rounding then touches only
    that small part, so Y1 and Y2 keep about the FP32 accuracy instead of the
    2^-9 relative accuracy of a BF16 product of Z itself."""
    m, n, r = 777, 640, 5
    say(f"mixed tangent_products, D = L + noise {noise:g}")
    rng = np.random.default_rng(4242)
    A = f32(rng.standard_normal((m, r)))
    B = f32(rng.standard_normal((n, r)) / np.sqrt(r))
    D = f32(A @ B.T + noise * rng.standard_normal((m, n)))
    Ut = f32(np.linalg.qr(rng.standard_normal((m, r)))[0])
    Vt = f32(np.linalg.qr(rng.standard_normal((n, r)))[0])
    zeta = 1e6   # S = 0, Z = D, E = D - L
    sv = R.Solver(dev(D, torch.float32), r, 0.01, 0.02, 0.5, 1.0, mixed=True)
    Y1, Y2, _ = sv.tangent_products(dev(A), dev(B), zeta, dev(Ut), dev(Vt))
    err = rel(Y1.cpu().numpy(), D @ Vt)
    err2 = rel(Y2.cpu().numpy(), D.T @ Ut)
    say(f"relative error of Y1 {err:.2e}, of Y2 {err2:.2e}")
    # BF16 rounding of E: ~2^-9 relative to |E| ~ noise, against |Y| ~ 1
    assert err < 4e-3 * noise + 2e-6, err
    assert err2 < 4e-3 * noise + 2e-6, err2


def _plain_and_mixed(x, mixed_err, tol=None, max_iter=100):
    D32 = dev(x.D, torch.float32)
    out = []
    for mixed in (False, True):
        sv = R.Solver(D32, x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol if tol is None else tol,
                      max_iter=max_iter, seed=7, mixed=mixed, mixed_err=mixed_err)
        R.rpca_profile_read_all()
        R.rpca_profile_enable(True)
        info = sv.solve()
        R.rpca_profile_enable(False)
        kinds = R.rpca_profile_read_all()
        U, s, V = (t.cpu().numpy() for t in sv.L_factors())
        out.append((info, (U * s) @ V.T, kinds))
    return out


def test_mixed_solve_config1_against_oracle_and_truth():
    x = I.config_instance(1, keep_L=True)
    say(f"mixed solve config 1: {x.m}x{x.n} r={x.r}")
    (ip, Lp, kp), (im, Lm, km) = _plain_and_mixed(x, 1e-3)
    assert ip.status == R.RPCA_OK and im.status == R.RPCA_OK
    assert im.err < x.tol
    assert im.iterations <= ip.iterations + 2
    # some bodies used the BF16 products, and the last ones the FP32 pass
    assert km[1][1] >= 1 and km[0][1] >= 1
    Do = f32(x.D)
    po = O.Params(r=x.r, beta=x.beta, beta_init=x.beta_init, gamma=x.gamma, mu=x.mu_in, tol=x.tol)
    res = O.solve(Do, po)
    assert rel(Lm, res.state.L()) <= 1e-4, rel(Lm, res.state.L())
    assert rel(Lm, x.L) <= 1e-4
    say(f"plain {ip.iterations} it, mixed {im.iterations} it, mixed vs oracle {rel(Lm, res.state.L()):.2e}")


def test_mixed_switch_levels():
    x = I.config_instance(1, keep_L=True)
    # a switch level above every err: only bodies 0 and 1 (enqueued before
    # any err is known) take BF16 products; err_0 is the FP32 residual
    (ip, Lp, kp), (im, Lm, km) = _plain_and_mixed(x, 10.0)
    assert km[1][1] == 2
    # (summed in another order by the other kernel: FP32 rounding apart)
    assert abs(im.err_hist[0] - ip.err_hist[0]) <= 1e-6 * ip.err_hist[0]
    assert abs(im.iterations - ip.iterations) <= 1
    assert rel(Lm, Lp) < 1e-4
    # and the decision is deterministic: the same solve twice, bitwise
    (_, _, _), (im2, Lm2, km2) = _plain_and_mixed(x, 1e-3)
    (_, _, _), (im3, Lm3, km3) = _plain_and_mixed(x, 1e-3)
    assert km2[1][1] == km3[1][1] and np.array_equal(Lm2, Lm3)
    assert np.array_equal(np.asarray(im2.err_hist), np.asarray(im3.err_hist))
    # a switch level below the tolerance (and the default, 0): every loop body
    # uses BF16 products, with FP32 residuals; since only the residual part
    # is rounded to BF16, the solve reaches the tolerance as the FP32 one does
    for level in (1e-12, 0.0):
        (ip, Lp, kp), (im, Lm, km) = _plain_and_mixed(x, level, max_iter=40)
        assert km[2][1] == im.init_passes          # the initialisation stays FP32
        assert km[0][1] == 0                        # and every loop pass was a BF16 one
        assert km[1][1] >= im.iterations
        assert im.status == R.RPCA_OK and im.err < x.tol
        assert abs(im.iterations - ip.iterations) <= 1
        assert rel(Lm, Lp) < 1e-5, rel(Lm, Lp)
        assert rel(Lm, x.L) <= 1e-4


@pytest.mark.parametrize("k", [1, 8])
def test_mixed_step_from_oracle_state(k):
    """One BF16-product body from the oracle's state k. Only the residual part
    E of Z = L_k + E is rounded to BF16 (8 bits per factor), so the error of
    Y1 is about 2^-8 |E| |V| and L_{k+1} moves by at most about
    2^-7 err_k ||D||_F / ||L_{k+1}||_F relative; late in a solve (k = 8,
    err_k ~ 1e-4) that is below the 1e-4 bar of the BF16 form."""
    x = I.config_instance(1, keep_L=True)
    Do = f32(x.D)
    po = O.Params(r=x.r, beta=x.beta, beta_init=x.beta_init, gamma=x.gamma, mu=x.mu_in, tol=x.tol)
    nD = O.frobenius(Do)
    st = O.initialize(Do, po, nD)
    for _ in range(k):
        st = O.step(Do, st, po, nD)
    nxt = O.step(Do, st, po, nD)
    sv = R.Solver(dev(x.D, torch.float32), x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol, mixed=True)
    sv.set_state(st.U, st.sigma, st.V, st.zeta, st.k, normD=nD)
    sv.step()
    U, s, V = (t.cpu().numpy() for t in sv.L_factors())
    d = rel((U * s) @ V.T, nxt.L())
    bound = 2.0 ** -7 * st.err * nD / np.linalg.norm(nxt.L()) + 1e-5
    say(f"mixed step from k={k}: err_k {st.err:.2e}, rel L {d:.2e}, bound {bound:.2e}")
    assert d <= bound
    assert abs(sv.state.zeta - nxt.zeta) / nxt.zeta <= bound
    if k >= 8:
        assert d <= 1e-4


def test_default_mixed_solve_against_oracle():
    """The default mixed form (BF16 E V in every loop body) against the FP64
    oracle directly: same iteration count and err trajectory, L within 1e-4."""
    x = I.config_instance(1, keep_L=True)
    Do = f32(x.D)
    po = O.Params(r=x.r, beta=x.beta, beta_init=x.beta_init, gamma=x.gamma, mu=x.mu_in, tol=x.tol)
    ref = O.solve(Do, po)
    sv = R.Solver(dev(x.D, torch.float32), x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol, seed=7,
                  mixed=True)
    info = sv.solve()
    U, s, V = (t.cpu().numpy() for t in sv.L_factors())
    d = rel((U * s) @ V.T, ref.state.L())
    say(f"default mixed solve: {info.iterations}/{ref.iterations} iterations, rel L {d:.2e}")
    assert info.status == R.RPCA_OK
    assert info.iterations == ref.iterations
    np.testing.assert_allclose(info.err_hist, ref.err_hist, rtol=1e-2)
    assert d <= 1e-4
    assert rel((U * s) @ V.T, x.L) <= 1e-4
