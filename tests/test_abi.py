"""C-ABI checks that need no GPU: the library loads, exports exactly what
include/rpca.h declares, and rejects invalid arguments before any launch."""
import ctypes
import os
import re

import pytest

from paper_1711_05519_amd import rpca as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpca.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*\**(rpca_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(R.LIB_PATH):
        pytest.skip("librpca.so not built")
    return R.library()


def test_header_and_exports_agree(lib):
    declared = _declared()
    assert set(declared) == set(R.EXPORTED), declared
    for name in declared:
        assert hasattr(lib, name), name


def test_struct_layout_matches_header(lib):
    # offsets the C compiler uses for the two structs (natural alignment)
    assert ctypes.sizeof(R.Params) == 8 * 3 + 4 * 2 + 8 * 5 + 4 * 4 + 8 + 8 + 8
    assert R.Params.zeta_mlp.offset == ctypes.sizeof(R.Params) - 8
    assert ctypes.sizeof(R.State) == 8 * 3 + 8 * 5 + 4 * 4


def _params(**kw):
    base = dict(m=100, n=80, ldd=80, r=3, dtype=R.RPCA_F64, beta=0.01, beta_init=0.02, gamma=0.5, mu=2.0,
                tol=1e-6, max_iter=100, init_block=0, init_max_passes=0, flags=0, seed=1)
    base.update(kw)
    return R.Params(**base)


def test_workspace_size_and_version(lib):
    assert lib.rpca_version() >= 100
    n = R.rpca_workspace_size(_params())
    assert n > 0 and n % 256 == 0
    # grows with the problem
    assert R.rpca_workspace_size(_params(m=1000, n=800, ldd=800)) > n
    assert lib.rpca_strerror(-1).decode() == "invalid argument"


@pytest.mark.parametrize("bad", [
    dict(m=0), dict(n=0), dict(ldd=79), dict(r=0), dict(r=17), dict(r=41), dict(dtype=7),
    dict(beta=0.0), dict(beta_init=-1.0), dict(gamma=1.0), dict(gamma=-0.1), dict(tol=0.0),
    dict(mu=0.0), dict(max_iter=-1), dict(init_block=2), dict(init_block=17), dict(flags=8),
    dict(beta=float("nan")), dict(tol=float("inf")),
    dict(flags=2, dtype=0), dict(flags=2, dtype=1, mixed_err=float("nan")), dict(flags=4, r=11, m=300, n=300, ldd=300),
    dict(flags=8), dict(flags=16),
])
def test_invalid_params_rejected(lib, bad):
    with pytest.raises(R.RpcaError) as e:
        R.rpca_workspace_size(_params(**bad))
    assert e.value.status == -1


def test_no_trim_allows_zero_mu(lib):
    assert R.rpca_workspace_size(_params(mu=0.0, flags=R.RPCA_FLAG_NO_TRIM)) > 0


def test_mixed_form_needs_fp32(lib):
    assert R.rpca_workspace_size(_params(dtype=R.RPCA_F32, flags=R.RPCA_FLAG_MIXED)) > 0
    assert R.rpca_workspace_size(_params(dtype=R.RPCA_F32, flags=R.RPCA_FLAG_MIXED | R.RPCA_FLAG_NO_TRIM,
                                         mu=0.0, mixed_err=1e-2)) > 0


def test_null_pointers_rejected_before_launch(lib):
    p = _params()
    st = R.State()
    ws = ctypes.create_string_buffer(16)
    assert lib.rpca_init(None, ctypes.byref(p), ctypes.byref(st), ws, 16, None) == -1
    assert lib.rpca_step(None, ctypes.byref(p), ctypes.byref(st), ws, 16, None) == -1
    assert lib.rpca_solve(None, ctypes.byref(p), ctypes.byref(st), None, None, 0, ws, 16, None) == -1
    # state without buffers
    d = ctypes.c_double(0)
    assert lib.rpca_init(ctypes.byref(d), ctypes.byref(p), ctypes.byref(st), ws, 16, None) == -1
    assert lib.rpca_trim(ctypes.byref(p), ctypes.byref(st), None, None, ws, 16, None) == -1


def test_training_workspace_is_larger(lib):
    base = R.rpca_workspace_size(_params(m=1000, n=900, ldd=900))
    assert R.rpca_workspace_size(_params(m=1000, n=900, ldd=900, flags=R.RPCA_FLAG_TRAINING)) > base


def test_relaxed_step_validates_before_launch(lib):
    p = _params(flags=R.RPCA_FLAG_TRAINING)
    st = R.State()
    out = R.RelaxResult()
    d = ctypes.c_double(0)
    ws = ctypes.create_string_buffer(16)
    # state without buffers, then missing factors: rejected before any device work
    assert lib.rpca_relaxed_step(ctypes.byref(d), ctypes.byref(p), ctypes.byref(st), 1.0, 0.1,
                                 ctypes.byref(d), ctypes.byref(d), 1, ctypes.byref(out), ws, 16, None) == -1
    st.U = st.V = st.sigma = ctypes.addressof(d)
    assert lib.rpca_relaxed_step(ctypes.byref(d), ctypes.byref(p), ctypes.byref(st), 1.0, 0.1,
                                 None, None, 1, ctypes.byref(out), ws, 16, None) == -1
    for zeta, tau, rt in [(0.0, 0.1, 1), (1.0, 0.0, 1), (float("nan"), 0.1, 1), (1.0, 0.1, 0), (1.0, 0.1, 17)]:
        assert lib.rpca_relaxed_step(ctypes.byref(d), ctypes.byref(p), ctypes.byref(st), zeta, tau,
                                     ctypes.byref(d), ctypes.byref(d), rt, ctypes.byref(out), ws, 16, None) == -1
    p2 = _params()   # no training workspace
    assert lib.rpca_relaxed_step(ctypes.byref(d), ctypes.byref(p2), ctypes.byref(st), 1.0, 0.1,
                                 ctypes.byref(d), ctypes.byref(d), 1, ctypes.byref(out), ws, 16, None) == -1


def test_mlp_entry_points_validate_before_launch(lib):
    ws = ctypes.create_string_buffer(64)
    assert lib.rpca_mlp_forward(None, ws, 1, ws, None) == -1
    assert lib.rpca_mlp_forward(ws, ws, -1, ws, None) == -1
    assert lib.rpca_mlp_backward(ws, ws, None, 1, ws, None) == -1
    assert lib.rpca_mlp_adam(ws, ws, ws, ws, 0, 0.1, 0.9, 0.999, 1e-8, None) == -1
    assert lib.rpca_mlp_adam(ws, ws, ws, ws, 1, 0.1, 1.0, 0.999, 1e-8, None) == -1


def test_solve_many_argument_checks(lib):
    # rejected before any device work: negative count, stream counts out of range
    f = lib.rpca_solve_many
    st = (ctypes.c_int32 * 1)()
    vp = (ctypes.c_void_p * 1)()
    for count, ns in ((-1, 1), (0, 0), (0, R.RPCA_MANY_MAX_STREAMS + 1)):
        assert f(count, None, None, None, None, None, 0, None, None, vp, ns, st) == R.RPCA_EINVAL
