"""Several solves advanced together (rpca_solve_many) against the same solves
run one by one (rpca_solve): every instance's result must be identical bit for
bit (the kernels are deterministic and each instance has its own workspace and
stream), including FP64 and FP32 instances, the mixed form and the learned
threshold side by side, more instances than streams, and an empty batch."""
import os

import numpy as np
import pytest
import torch

from paper_1711_05519_amd import inputs as I
from paper_1711_05519_amd import learn as LN
from paper_1711_05519_amd import rpca as R

pytestmark = pytest.mark.gpu


def make(spec):
    m, n, r, alpha, dtype, kw, seed = spec
    x = I.gaussian_instance(m, n, r, alpha, 1.0, seed=seed, tol=1e-5 if dtype == torch.float32 else 1e-7)
    D = torch.as_tensor(x.D, dtype=dtype, device="cuda")
    return R.Solver(D, r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol, seed=3, **kw)


def specs():
    theta = LN.load_theta(os.path.join(os.path.dirname(LN.__file__), "zeta_mlp.npy"))
    return [(300, 250, 3, 0.1, torch.float64, {}, 11), (500, 400, 4, 0.2, torch.float32, {}, 12),
            (640, 700, 5, 0.1, torch.float32, {"mixed": True}, 13), (800, 800, 6, 0.15, torch.float32,
                                                                      {"learned": theta}, 14),
            (257, 513, 2, 0.05, torch.float64, {"trim": False}, 15), (1000, 1000, 5, 0.1, torch.float32, {}, 16)]


def test_solve_many_matches_one_by_one():
    sp = specs()
    ref = []
    for s in sp:
        sv = make(s)
        info = sv.solve()
        ref.append((info, sv.U.clone(), sv.V.clone(), sv.sigma.clone()))
    svs = [make(s) for s in sp]
    infos = R.solve_many(svs, n_streams=3)
    for (ri, U, V, sg), sv, info in zip(ref, svs, infos):
        assert info.status == ri.status == R.RPCA_OK
        assert info.iterations == ri.iterations and info.init_passes == ri.init_passes
        assert info.err_hist == ri.err_hist and info.zeta_hist == ri.zeta_hist
        assert torch.equal(sv.U, U) and torch.equal(sv.V, V) and torch.equal(sv.sigma, sg)


def test_solve_many_one_stream_and_empty_batch():
    sp = specs()[:3]
    svs = [make(s) for s in sp]
    infos = R.solve_many(svs, n_streams=1)
    assert all(i.status == R.RPCA_OK for i in infos)
    assert R.rpca_solve_many([], [], [], None, None, [], [torch.cuda.Stream()]) == []


def test_solve_many_rejects_a_bad_instance_before_running():
    sp = specs()[:2]
    svs = [make(s) for s in sp]
    svs[1].params.gamma = 1.5    # invalid
    k0 = svs[0].state.k
    with pytest.raises(R.RpcaError) as e:
        R.solve_many(svs, n_streams=2)
    assert e.value.status == R.RPCA_EINVAL
    assert svs[0].state.k == k0   # nothing ran
