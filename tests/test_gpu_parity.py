"""HIP path against the FP64 oracle, element by element on identical inputs.

Tolerances (relative Frobenius unless stated): FP64 path 1e-10, FP32 path
1e-5 for L; the support of S must agree except for entries whose |x| lies
within the same tolerance (scaled by max|D|) of zeta.
For the FP32 path the oracle runs in FP64 on the FP32-rounded D (and on
FP32-rounded inputs where the library rounds its inputs), so the comparison
isolates the library's arithmetic.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1711_05519_amd import inputs as I
from paper_1711_05519_amd import rpca as R

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}
DT = [torch.float64, torch.float32]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def as_seen(D, dtype):
    """D as the library sees it, promoted to FP64 for the oracle."""
    return D.astype(np.float32).astype(np.float64) if dtype == torch.float32 else D.copy()


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def oparams(x, tol=None, mu=None, max_iter=100):
    return O.Params(r=x.r, beta=x.beta, beta_init=x.beta_init, gamma=x.gamma,
                    mu=x.mu_in if mu is None else mu, tol=x.tol if tol is None else tol, max_iter=max_iter)


def solver(x, dtype, tol=None, trim=True, max_iter=100, init_block=0, D=None):
    Dd = dev(x.D if D is None else D, dtype)
    return R.Solver(Dd, x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol if tol is None else tol,
                    max_iter=max_iter, trim=trim, init_block=init_block, seed=7)


def L_of(U, s, V):
    return (np.asarray(U) * np.asarray(s)) @ np.asarray(V).T


def gpu_L(sv):
    U, s, V = (t.cpu().numpy() for t in sv.L_factors())
    return L_of(U, s, V)


def support_agrees(D, L_ref, zeta_ref, S_gpu, tol):
    x = D - L_ref
    margin = tol * max(1.0, np.abs(D).max()) * 10
    ambiguous = np.abs(np.abs(x) - zeta_ref) <= margin
    ref = np.abs(x) > zeta_ref
    got = S_gpu != 0
    bad = (ref != got) & ~ambiguous
    return int(bad.sum()), int(ambiguous.sum())


# ------------------------------------------------------- dominant pass ----

def _zeta_with_margin(x, q, margin):
    a = np.sort(np.abs(x).reshape(-1))
    i = int(q * a.size)
    while i + 1 < a.size and a[i + 1] - a[i] <= 2 * margin:
        i += 1
    return 0.5 * (a[i] + a[i + 1])


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("m,n,r", [(300, 270, 3), (64, 520, 1), (1031, 259, 5), (200, 200, 16)])
def test_tangent_products(dtype, m, n, r):
    say(f"tangent_products dtype={dtype} m={m} n={n} r={r}")
    rng = np.random.default_rng(m + n + r)
    D = rng.standard_normal((m, n)) * 2.0
    A = rng.standard_normal((m, r))
    B = rng.standard_normal((n, r)) / np.sqrt(r)
    Ut, _ = np.linalg.qr(rng.standard_normal((m, r)))
    Vt, _ = np.linalg.qr(rng.standard_normal((n, r)))
    cast = (lambda a: a.astype(np.float32).astype(np.float64)) if dtype == torch.float32 else (lambda a: a)
    Do, Ao, Bo, Uo, Vo = map(cast, (D, A, B, Ut, Vt))
    x = Do - Ao @ Bo.T
    zeta = _zeta_with_margin(x, 0.8, 1e-4 * np.abs(x).max())
    S = O.hard_threshold(x, zeta)
    Z = Do - S
    Y1o, Y2o = Z @ Vo, Z.T @ Uo
    res_o = float(np.sum(np.where(np.abs(x) <= zeta, x * x, 0.0)))
    Dd = dev(D, dtype)
    sv = R.Solver(Dd, r, 0.01, 0.02, 0.5, 1.0)
    Y1, Y2, res = sv.tangent_products(dev(A), dev(B), zeta, dev(Ut), dev(Vt))
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    assert rel(Y1.cpu().numpy(), Y1o) < tol
    assert rel(Y2.cpu().numpy(), Y2o) < tol
    assert abs(res - res_o) / res_o < tol


@pytest.mark.parametrize("dtype", DT)
def test_tangent_products_edge_thresholds(dtype):
    # zeta = +inf: S = 0, resid = ||D - L||^2 ; zeta < 0: S = D - L, Z = L, resid = 0
    rng = np.random.default_rng(3)
    m, n, r = 130, 300, 2
    D = rng.standard_normal((m, n))
    A, B = rng.standard_normal((m, r)), rng.standard_normal((n, r))
    Ut, _ = np.linalg.qr(rng.standard_normal((m, r)))
    Vt, _ = np.linalg.qr(rng.standard_normal((n, r)))
    sv = R.Solver(dev(D, dtype), r, 0.01, 0.02, 0.5, 1.0)
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    Y1, Y2, res = sv.tangent_products(dev(A), dev(B), float("inf"), dev(Ut), dev(Vt))
    x = D - A @ B.T
    assert abs(res - np.sum(x * x)) / np.sum(x * x) < tol
    assert rel(Y1.cpu().numpy(), D @ Vt) < tol
    Y1, Y2, res = sv.tangent_products(dev(A), dev(B), -1.0, dev(Ut), dev(Vt))
    assert res == 0.0
    assert rel(Y1.cpu().numpy(), (A @ B.T) @ Vt) < (1e-12 if dtype == torch.float64 else 1e-5)


# ----------------------------------------------------------------- trim ---

@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("m,n,r", [(500, 300, 4), (257, 700, 2)])
def test_trim_matches_oracle(dtype, m, n, r):
    say(f"trim dtype={dtype} m={m} n={n} r={r}")
    rng = np.random.default_rng(11 * m + n)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    U[:5] *= 8.0
    V[3] *= 10.0
    U, _ = np.linalg.qr(U)
    V, _ = np.linalg.qr(V)
    s = np.sort(rng.uniform(1, 10, r))[::-1]
    mu = 1.5
    D = rng.standard_normal((m, n))
    sv = R.Solver(dev(D, dtype), r, 0.01, 0.02, 0.5, mu)
    sv.set_state(U, s, V, zeta=1.0, k=0)
    Ut, Vt = sv.trim()
    Uo, Vo = O.trimmed_bases(U, V, mu, r)
    Ut, Vt = Ut.cpu().numpy(), Vt.cpu().numpy()
    assert np.abs(Ut.T @ Ut - np.eye(r)).max() < 1e-13
    assert np.abs(Vt.T @ Vt - np.eye(r)).max() < 1e-13
    assert rel(Ut @ Ut.T, Uo @ Uo.T) < 1e-12
    assert rel(Vt @ Vt.T, Vo @ Vo.T) < 1e-12


# ---------------------------------------------------------------- step ----

def _oracle_state_after(x, D, p, k):
    st = O.initialize(D, p)
    for _ in range(k):
        st = O.step(D, st, p)
    return st


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("m,n,r,alpha,c,k,trim", [
    (400, 300, 4, 0.1, 1.0, 5, True),
    (333, 517, 3, 0.2, 2.0, 3, True),
    (300, 300, 5, 0.1, 1.0, 6, False),
    # either side of m + n = 8192, where the gather switches from 64-row to 128-row workgroups
    (7992, 200, 3, 0.1, 1.0, 3, True),
    (7993, 200, 3, 0.1, 1.0, 3, True),
])
def test_step_from_oracle_state(dtype, m, n, r, alpha, c, k, trim):
    say(f"step dtype={dtype} m={m} n={n} r={r} k={k} trim={trim}")
    x = I.gaussian_instance(m, n, r, alpha, c, seed=m * 7 + n + k)
    D = as_seen(x.D, dtype)
    p = oparams(x, mu=x.mu_in if trim else 0.0)
    st = _oracle_state_after(x, D, p, k)
    nxt = O.step(D, st, p)
    sv = solver(x, dtype, trim=trim)
    sv.set_state(st.U, st.sigma, st.V, st.zeta, st.k, normD=np.linalg.norm(D))
    sv.step()
    tol = TOL[dtype]
    L_gpu, L_ref = gpu_L(sv), nxt.L()
    say(f"  rel L {rel(L_gpu, L_ref):.3e} zeta {sv.state.zeta:.6g}/{nxt.zeta:.6g} err {sv.state.err:.6e}/{nxt.err:.6e}")
    assert rel(L_gpu, L_ref) <= tol
    assert abs(sv.state.zeta - nxt.zeta) <= tol * nxt.zeta
    assert abs(sv.state.err - nxt.err) <= 10 * tol * max(nxt.err, 1e-3)
    assert sv.state.k == st.k + 1
    np.testing.assert_allclose(sv.sigma.cpu().numpy(), nxt.sigma, rtol=tol)
    _, S = sv.materialize(want_L=False)
    bad, amb = support_agrees(D, L_ref, nxt.zeta, S.cpu().numpy(), tol)
    assert bad == 0, (bad, amb)


# ---------------------------------------------------------------- init ----

@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("m,n,r,alpha,c,bi_scale", [
    (500, 400, 5, 0.1, 1.0, 1.0),
    (300, 650, 2, 0.15, 5.0, 0.3),    # S_{-1} non-empty
])
def test_init_matches_oracle(dtype, m, n, r, alpha, c, bi_scale):
    say(f"init dtype={dtype} m={m} n={n} r={r}")
    x = I.gaussian_instance(m, n, r, alpha, c, seed=100 + m + n)
    x.beta_init *= bi_scale
    D = as_seen(x.D, dtype)
    p = oparams(x)
    st, tr = O.initialize(D, p, trace=True)
    sv = solver(x, dtype)
    sv.init()
    tol = TOL[dtype]
    L_gpu = gpu_L(sv)
    say(f"  rel L0 {rel(L_gpu, st.L()):.3e} passes {sv.state.init_passes} zeta0 {sv.state.zeta}/{st.zeta}")
    assert rel(L_gpu, st.L()) <= tol
    assert abs(sv.state.zeta - st.zeta) <= tol * st.zeta
    assert abs(sv.state.err - st.err) <= 10 * tol * st.err
    assert abs(sv.state.normD - np.linalg.norm(D)) <= 1e-12 * np.linalg.norm(D) if dtype == torch.float64 else True


# --------------------------------------------------------------- solve ----

@pytest.mark.parametrize("dtype", DT)
def test_solve_config1(dtype):
    say(f"solve config1 dtype={dtype}")
    x = I.config_instance(1)
    tol_solve = 1e-6 if dtype == torch.float64 else 1e-5
    D = as_seen(x.D, dtype)
    res_o = O.solve(D, oparams(x, tol=tol_solve))
    sv = solver(x, dtype, tol=tol_solve)
    info = sv.solve()
    L_gpu = gpu_L(sv)
    say(f"  iters {info.iterations}/{res_o.iterations} err {info.err:.3e}/{res_o.state.err:.3e} "
        f"relL {rel(L_gpu, res_o.state.L()):.3e} recovery {O.recovery_error(L_gpu, x.L):.2e}")
    assert info.status == R.RPCA_OK
    assert info.iterations == res_o.iterations
    np.testing.assert_allclose(info.err_hist, res_o.err_hist, rtol=1e-8 if dtype == torch.float64 else 1e-3)
    assert rel(L_gpu, res_o.state.L()) <= TOL[dtype]
    assert O.recovery_error(L_gpu, x.L) <= 1e-4          # success criterion of Section 3


def test_solve_is_deterministic():
    x = I.gaussian_instance(600, 500, 4, 0.1, 1.0, seed=5, tol=1e-5)
    a = solver(x, torch.float32)
    ia = a.solve()
    b = solver(x, torch.float32)
    ib = b.solve()
    assert ia.err_hist == ib.err_hist
    assert torch.equal(a.U, b.U) and torch.equal(a.V, b.V) and torch.equal(a.sigma, b.sigma)


def test_max_iter_status():
    x = I.gaussian_instance(300, 300, 3, 0.1, 1.0, seed=6)
    sv = solver(x, torch.float64, tol=1e-14, max_iter=3)
    info = sv.solve()
    assert info.status == R.RPCA_MAXITER and info.iterations == 3


def test_histories_short_and_long():
    """The last kernel of a solve copies the control block and the leading 128
    entries of both histories into mapped host memory; a longer history is
    read with copies. A slow threshold decay (gamma = 0.9) and an unreachable
    tol run 140 iterations (141 entries); the same solve capped at 100
    iterations must give the same leading entries bit for bit, and both follow
    the FP64 oracle while err is well above the rounding level."""
    x = I.gaussian_instance(200, 180, 3, 0.1, 1.0, seed=6)
    say("histories: 200x180 r=3 gamma=0.9, 140 and 100 iterations")
    D = dev(x.D, torch.float64)
    run = {}
    for it in (140, 100):
        sv = R.Solver(D, x.r, x.beta, x.beta_init, 0.9, x.mu_in, tol=1e-300, max_iter=it, seed=7)
        run[it] = sv.solve()
        info = run[it]
        assert info.status == R.RPCA_MAXITER and info.iterations == it
        assert len(info.err_hist) == len(info.zeta_hist) == it + 1
        assert info.err_hist[-1] == info.err
    a, b = run[140], run[100]
    assert a.err_hist[:101] == b.err_hist and a.zeta_hist[:101] == b.zeta_hist
    p = O.Params(r=x.r, beta=x.beta, beta_init=x.beta_init, gamma=0.9, mu=x.mu_in, tol=1e-300, max_iter=140)
    ref = O.solve(x.D, p)
    assert ref.iterations == 140
    eo = np.asarray(ref.err_hist)
    above = eo > 1e-8
    say(f"  {int(above.sum())} entries above 1e-8; err_140 {a.err:.2e} (oracle {eo[-1]:.2e})")
    np.testing.assert_allclose(np.asarray(a.err_hist)[above], eo[above], rtol=1e-6)
    np.testing.assert_allclose(a.zeta_hist[:20], ref.zeta_hist[:20], rtol=1e-8, atol=2e-8 * ref.zeta_hist[1] / 0.9)
    assert a.err < 1e-12


def test_history_cap_and_null_histories():
    """hist_cap below the iteration count: exactly hist_cap entries are
    written (the rest of the caller's arrays stays untouched) and equal the
    full histories' leading entries; null histories are accepted."""
    import ctypes
    x = I.gaussian_instance(300, 260, 3, 0.1, 1.0, seed=8)
    say("history cap: 300x260 r=3")
    sv = solver(x, torch.float32, tol=1e-5)
    full = sv.solve()
    assert full.iterations >= 5
    lib = R._lib()
    for cap in (3, 1, 0):
        eh = (ctypes.c_double * 8)(*([-7.0] * 8))
        zh = (ctypes.c_double * 8)(*([-7.0] * 8))
        rc = lib.rpca_solve(R._ptr(sv.D), ctypes.byref(sv.params), ctypes.byref(sv.state), eh, zh, cap,
                            *R._ws(sv.ws), R._stream(None))
        assert rc == R.RPCA_OK and sv.state.k == full.iterations
        assert list(eh[:cap]) == full.err_hist[:cap] and list(zh[:cap]) == full.zeta_hist[:cap]
        assert list(eh[cap:]) == [-7.0] * (8 - cap) and list(zh[cap:]) == [-7.0] * (8 - cap)
    rc = lib.rpca_solve(R._ptr(sv.D), ctypes.byref(sv.params), ctypes.byref(sv.state), None, None, 8,
                        *R._ws(sv.ws), R._stream(None))
    assert rc == R.RPCA_OK and sv.state.k == full.iterations and sv.state.err == full.err


# ---------------------------------------------------------- edge cases ----

def test_unaligned_leading_dimension_matches_contiguous():
    x = I.gaussian_instance(300, 257, 3, 0.1, 1.0, seed=9, tol=1e-5)
    base = torch.zeros((300, 258), dtype=torch.float32, device="cuda")
    base[:, :257] = dev(x.D, torch.float32)
    Dv = base[:, :257]            # row stride 258 floats: rows are not 16-byte aligned
    a = R.Solver(Dv, x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=1e-5, seed=7)
    ia = a.solve()
    b = solver(x, torch.float32, tol=1e-5)
    ib = b.solve()
    assert ia.err_hist == ib.err_hist
    assert torch.equal(a.U, b.U)


def test_exactly_low_rank_input():
    # S = 0 and zeta_{-1} above every |D_ij|: L_0 = D, the complements W1, W2
    # vanish and the Cholesky factors of their Grams degenerate.
    rng = np.random.default_rng(2)
    m, n, r = 200, 150, 3
    D = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    p = O.Params(r=r, beta=0.05, beta_init=0.1, gamma=0.5, mu=5.0, tol=1e-12, max_iter=3)
    ref = O.solve(D, p, fixed_iters=3)
    sv = R.Solver(dev(D), r, 0.05, 0.1, 0.5, 5.0, tol=1e-12, max_iter=5)
    info = sv.solve()
    assert info.err < 1e-12
    assert rel(gpu_L(sv), D) < 1e-12
    # three forced steps from L_0 = D stay at D
    sv.set_state(ref.state.U, ref.state.sigma, ref.state.V, ref.state.zeta, 0, normD=np.linalg.norm(D))
    for _ in range(3):
        sv.step()
    assert rel(gpu_L(sv), D) < 1e-12


@pytest.mark.parametrize("m,n,r,p", [(8, 8, 2, 4), (40, 33, 1, 0), (64, 300, 16, 16), (3000, 40, 2, 0)])
def test_shapes_run_and_match_oracle_step(m, n, r, p):
    say(f"shape m={m} n={n} r={r} p={p}")
    x = I.gaussian_instance(m, n, r, 0.05, 1.0, seed=m * n + r)
    D = x.D
    po = oparams(x)
    st = O.initialize(D, po)
    sv = R.Solver(dev(D), r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=1e-8, init_block=p, seed=3)
    sv.init()
    assert rel(gpu_L(sv), st.L()) <= 1e-9
    nxt = O.step(D, st, po)
    sv.set_state(st.U, st.sigma, st.V, st.zeta, st.k, normD=np.linalg.norm(D))
    sv.step()
    assert rel(gpu_L(sv), nxt.L()) <= 1e-9
