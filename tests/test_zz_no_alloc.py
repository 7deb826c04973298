"""rpca_step_noalloc (the variant of rpca_step for callers that cannot
allocate: its workspace is the library's own per-GPU buffer) against
rpca_step with a caller workspace, through the C ABI: two calls in a row, the
second on a smaller problem, each bit for bit equal to rpca_step from the
same state; and a problem too large for the buffer is refused before any
launch."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1711_05519_amd import inputs as I
from paper_1711_05519_amd import rpca as R

pytestmark = pytest.mark.gpu


def _case(m, n, r, seed, dtype):
    x = I.gaussian_instance(m, n, r, 0.1, 1.0, seed=seed)
    D = x.D.astype(np.float32).astype(np.float64) if dtype == torch.float32 else x.D
    p = O.Params(r=r, beta=x.beta, beta_init=x.beta_init, gamma=x.gamma, mu=x.mu_in, tol=1e-8)
    st = O.step(D, O.initialize(D, p), p)       # a state one iteration in
    Dd = torch.as_tensor(D, dtype=dtype, device="cuda")
    svs = []
    for _ in range(2):
        sv = R.Solver(Dd, r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=1e-8)
        sv.set_state(st.U, st.sigma, st.V, st.zeta, st.k, normD=np.linalg.norm(D))
        svs.append(sv)
    return svs


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_step_matches_step_twice(dtype):
    for (m, n, r, seed) in [(700, 600, 4, 1), (300, 260, 3, 2)]:     # the second call is smaller
        a, b = _case(m, n, r, seed, dtype)
        print(f"noalloc step {m}x{n} r={r} {dtype}", flush=True)
        a.step()
        b.step_noalloc()
        torch.cuda.synchronize()
        assert torch.equal(a.U, b.U) and torch.equal(a.V, b.V) and torch.equal(a.sigma, b.sigma)
        assert (a.state.k, a.state.zeta, a.state.err) == (b.state.k, b.state.zeta, b.state.err)
        # and a second step of each from there
        a.step()
        b.step_noalloc()
        assert torch.equal(a.U, b.U) and a.state.err == b.state.err


def test_noalloc_refuses_a_problem_larger_than_its_buffer():
    D = torch.zeros((1, 1), dtype=torch.float32, device="cuda")
    p = R.Params(m=20000, n=20000, ldd=20000, r=10, dtype=R.RPCA_F32, beta=0.01, beta_init=0.02, gamma=0.5,
                 mu=2.0, tol=1e-6, max_iter=100, init_block=0, init_max_passes=0, flags=0, seed=1)
    assert R.rpca_workspace_size(p) > R.RPCA_NOALLOC_WS_BYTES
    U = torch.zeros((20000, 10), dtype=torch.float64, device="cuda")
    s = torch.ones((10,), dtype=torch.float64, device="cuda")
    st = R.State(U=U.data_ptr(), V=U.data_ptr(), sigma=s.data_ptr(), zeta=1.0, err=float("nan"), sigma1_pt=0.0,
                 sigma_r1_pt=0.0, normD=1.0, k=0, init_passes=0)
    with pytest.raises(R.RpcaError) as e:
        R.rpca_step_noalloc(D, p, st)
    assert e.value.status == R.RPCA_EWORKSPACE
    assert st.k == 0
