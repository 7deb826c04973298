"""RPCA_TRACE: per-state JSON lines of finished solves (a file named by the
variable), equal to the histories the solve returns."""
import json
import os

import pytest
import torch

from paper_1711_05519_amd import inputs as I
from paper_1711_05519_amd import rpca as R

pytestmark = pytest.mark.gpu


def test_trace_lines_match_the_histories(tmp_path):
    path = tmp_path / "trace.jsonl"
    x = I.gaussian_instance(300, 260, 3, 0.1, 1.0, seed=61, tol=1e-5)
    D = torch.as_tensor(x.D, dtype=torch.float32, device="cuda")
    old = os.environ.get("RPCA_TRACE")
    os.environ["RPCA_TRACE"] = str(path)
    try:
        sv = R.Solver(D, x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol, seed=7)
        info = sv.solve()
        bs = R.BatchSolver(torch.stack([D, D]), x.r, x.beta, x.beta_init, x.gamma, x.mu_in, tol=x.tol, seed=7)
        binfo = bs.solve()
    finally:
        if old is None:
            del os.environ["RPCA_TRACE"]
        else:
            os.environ["RPCA_TRACE"] = old
    lines = [json.loads(l) for l in path.read_text().splitlines()]
    single = [l for l in lines if l["call"] == "rpca_solve"]
    steps = [l for l in single if "k" in l and "status" not in l]
    assert [l["k"] for l in steps] == list(range(info.iterations + 1))
    assert [l["err"] for l in steps] == info.err_hist
    assert [l["zeta"] for l in steps] == info.zeta_hist
    summary = [l for l in single if "status" in l]
    assert len(summary) == 1 and summary[0]["iterations"] == info.iterations and summary[0]["status"] == info.status
    batch = [l for l in lines if l["call"] == "rpca_solve_batch" and "status" in l]
    assert [b["instance"] for b in batch] == [0, 1]
    assert all(b["iterations"] == i.iterations for b, i in zip(batch, binfo))
    for i, bi in enumerate(binfo):
        errs = [l["err"] for l in lines if l["call"] == "rpca_solve_batch" and l["instance"] == i and "status" not in l]
        assert errs == bi.err_hist
