"""Thin Python binding of librpca (include/rpca.h).

Argument marshalling only: every computation runs in the HIP library. Device
buffers are torch CUDA tensors (ROCm build), passed by data pointer together
with torch's current stream. The functions keep the C names:

    rpca_workspace_size, rpca_init, rpca_trim, rpca_step, rpca_solve,
    rpca_materialize, rpca_tangent_products

`Solver` bundles the parameter struct, the iterate buffers and the workspace.
There is no fallback: if the library is missing or no gfx950 device is
current, calls raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpca.so")

RPCA_OK, RPCA_MAXITER = 0, 1
RPCA_EINVAL, RPCA_EWORKSPACE, RPCA_EHIP, RPCA_ENODEV, RPCA_EBREAKDOWN = -1, -2, -3, -4, -5
RPCA_F64, RPCA_F32 = 0, 1
RPCA_FLAG_NO_TRIM = 1
RPCA_FLAG_MIXED = 2
RPCA_FLAG_TRAINING = 4
RPCA_FLAG_LEARNED = 8
RPCA_MLP_PARAMS = 1249
RPCA_PROF_KINDS = 4
RPCA_MAX_RANK = 16

EXPORTED = ("rpca_workspace_size", "rpca_init", "rpca_trim", "rpca_step", "rpca_step_noalloc", "rpca_solve",
            "rpca_solve_many",
            "rpca_materialize", "rpca_tangent_products", "rpca_strerror",
            "rpca_last_hip_error", "rpca_version", "rpca_profile_enable", "rpca_profile_read",
            "rpca_relaxed_step", "rpca_unrolled_adjoint", "rpca_batch_layout_of", "rpca_solve_batch",
            "rpca_mlp_forward", "rpca_mlp_backward", "rpca_mlp_adam", "rpca_read_probe")


class RpcaError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib().rpca_strerror(status).decode()
        if status == -3:
            msg += f" (hipError {_lib().rpca_last_hip_error()})"
        super().__init__(f"{where}: {msg} [status {status}]")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("ldd", ctypes.c_int64),
                ("r", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("beta", ctypes.c_double), ("beta_init", ctypes.c_double), ("gamma", ctypes.c_double),
                ("mu", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("init_block", ctypes.c_int32),
                ("init_max_passes", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("mixed_err", ctypes.c_double), ("zeta_mlp", ctypes.c_void_p)]


class State(ctypes.Structure):
    _fields_ = [("U", ctypes.c_void_p), ("V", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("zeta", ctypes.c_double), ("err", ctypes.c_double),
                ("sigma1_pt", ctypes.c_double), ("sigma_r1_pt", ctypes.c_double),
                ("normD", ctypes.c_double), ("k", ctypes.c_int32), ("init_passes", ctypes.c_int32),
                ("svd_sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchLayout(ctypes.Structure):
    _fields_ = [("slab_bytes", ctypes.c_size_t), ("off_D", ctypes.c_size_t), ("off_U", ctypes.c_size_t),
                ("off_V", ctypes.c_size_t), ("off_sigma", ctypes.c_size_t), ("off_ws", ctypes.c_size_t)]


class RelaxResult(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_double), ("dloss_dzeta", ctypes.c_double), ("err", ctypes.c_double),
                ("sigma1", ctypes.c_double), ("sigma_r1", ctypes.c_double),
                ("svd_sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (python -m paper_1711_05519_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        P, S, vp, d = ctypes.POINTER(Params), ctypes.POINTER(State), ctypes.c_void_p, ctypes.c_double
        pd = ctypes.POINTER(ctypes.c_double)
        sz = ctypes.c_size_t
        sig = {
            "rpca_workspace_size": [P, ctypes.POINTER(sz)],
            "rpca_init": [vp, P, S, vp, sz, vp],
            "rpca_trim": [P, S, vp, vp, vp, sz, vp],
            "rpca_step": [vp, P, S, vp, sz, vp],
            "rpca_step_noalloc": [vp, P, S, vp],
            "rpca_solve": [vp, P, S, pd, pd, ctypes.c_int32, vp, sz, vp],
            "rpca_solve_many": [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(P), ctypes.POINTER(S),
                                ctypes.POINTER(pd), ctypes.POINTER(pd), ctypes.c_int32, ctypes.POINTER(vp),
                                ctypes.POINTER(sz), ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
            "rpca_materialize": [vp, P, S, vp, ctypes.c_int64, vp, ctypes.c_int64, vp, sz, vp],
            "rpca_tangent_products": [vp, P, vp, vp, d, vp, vp, vp, vp, pd, vp, sz, vp],
            "rpca_relaxed_step": [vp, P, S, d, d, vp, vp, ctypes.c_int32, ctypes.POINTER(RelaxResult), vp, sz, vp],
            "rpca_batch_layout_of": [P, ctypes.POINTER(BatchLayout)],
            "rpca_solve_batch": [ctypes.c_int32, vp, P, S, pd, pd, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), vp],
            "rpca_unrolled_adjoint": [vp, P, ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      pd, pd, pd, vp, vp, ctypes.c_int32, pd, vp, vp, vp, vp, sz, vp],
            "rpca_mlp_forward": [vp, vp, ctypes.c_int32, vp, vp],
            "rpca_read_probe": [vp, ctypes.c_int64, vp, vp],
            "rpca_mlp_backward": [vp, vp, vp, ctypes.c_int32, vp, vp],
            "rpca_mlp_adam": [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, vp],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        lib.rpca_strerror.argtypes = [ctypes.c_int]
        lib.rpca_strerror.restype = ctypes.c_char_p
        lib.rpca_last_hip_error.restype = ctypes.c_int
        lib.rpca_version.restype = ctypes.c_int
        lib.rpca_profile_enable.argtypes = [ctypes.c_int]
        lib.rpca_profile_enable.restype = ctypes.c_int
        lib.rpca_profile_read.argtypes = [pd, ctypes.POINTER(ctypes.c_int64)]
        lib.rpca_profile_read.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def library():
    """The loaded ctypes library (loads it on first use)."""
    return _lib()


def _check(status: int, where: str) -> int:
    if status < 0:
        raise RpcaError(status, where)
    return status


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ws(ws: torch.Tensor):
    return ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * ws.element_size())


# ---- the C entry points ------------------------------------------------------

def rpca_workspace_size(params: Params) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib().rpca_workspace_size(ctypes.byref(params), ctypes.byref(n)), "rpca_workspace_size")
    return int(n.value)


def rpca_init(D, params, state, ws, stream=None) -> int:
    w, nb = _ws(ws)
    return _check(_lib().rpca_init(_ptr(D), ctypes.byref(params), ctypes.byref(state), w, nb, _stream(stream)),
                  "rpca_init")


def rpca_trim(params, state, U_tilde, V_tilde, ws, stream=None) -> int:
    w, nb = _ws(ws)
    return _check(_lib().rpca_trim(ctypes.byref(params), ctypes.byref(state), _ptr(U_tilde), _ptr(V_tilde),
                                   w, nb, _stream(stream)), "rpca_trim")


def rpca_step(D, params, state, ws, stream=None) -> int:
    w, nb = _ws(ws)
    return _check(_lib().rpca_step(_ptr(D), ctypes.byref(params), ctypes.byref(state), w, nb, _stream(stream)),
                  "rpca_step")


RPCA_NOALLOC_WS_BYTES = 64 << 20


def rpca_step_noalloc(D, params, state, stream=None) -> int:
    """rpca_step with the library's own per-GPU workspace (allocates nothing)."""
    return _check(_lib().rpca_step_noalloc(_ptr(D), ctypes.byref(params), ctypes.byref(state), _stream(stream)),
                  "rpca_step_noalloc")


def rpca_relaxed_step(D, params, state, zeta, tau, P, Q, ws, stream=None) -> RelaxResult:
    """One relaxed iteration (see include/rpca.h); P, Q: FP64 device factors."""
    if P.dtype != torch.float64 or Q.dtype != torch.float64 or P.shape[1] != Q.shape[1]:
        raise ValueError("P and Q must be FP64 with the same number of columns")
    P, Q = P.contiguous(), Q.contiguous()
    out = RelaxResult()
    w, nb = _ws(ws)
    _check(_lib().rpca_relaxed_step(_ptr(D), ctypes.byref(params), ctypes.byref(state), float(zeta), float(tau),
                                    _ptr(P), _ptr(Q), int(P.shape[1]), ctypes.byref(out), w, nb, _stream(stream)),
           "rpca_relaxed_step")
    return out


RPCA_MAX_UNROLL = 64


def rpca_unrolled_adjoint(D, params, Us, ss, Vs, zetas, taus, weights, P, Q, U_bar, s_bar, V_bar, ws,
                          stream=None) -> np.ndarray:
    """Reverse mode of K unrolled relaxed iterations (see include/rpca.h).
    Us, ss, Vs: the K + 1 checkpoints (FP64 device tensors); zetas, taus,
    weights: K values; P, Q: FP64 device target factors; U_bar, s_bar, V_bar:
    FP64 device outputs. Returns d loss / d zeta_k (K values)."""
    K = len(zetas)
    if not (len(Us) == len(ss) == len(Vs) == K + 1 and len(taus) == K and len(weights) == K):
        raise ValueError("K + 1 checkpoints and K thresholds, temperatures and weights are required")
    if P.dtype != torch.float64 or Q.dtype != torch.float64 or P.shape[1] != Q.shape[1]:
        raise ValueError("P and Q must be FP64 with the same number of columns")
    for t in list(Us) + list(ss) + list(Vs) + [U_bar, s_bar, V_bar]:
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("checkpoints and outputs must be contiguous FP64 device tensors")
    P, Q = P.contiguous(), Q.contiguous()
    arr = lambda ts: (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])
    dbl = lambda xs: (ctypes.c_double * len(xs))(*[float(x) for x in xs])
    zb = (ctypes.c_double * K)()
    w, nb = _ws(ws)
    _check(_lib().rpca_unrolled_adjoint(_ptr(D), ctypes.byref(params), K, arr(Us), arr(ss), arr(Vs), dbl(zetas),
                                        dbl(taus), dbl(weights), _ptr(P), _ptr(Q), int(P.shape[1]), zb,
                                        _ptr(U_bar), _ptr(s_bar), _ptr(V_bar), w, nb, _stream(stream)),
           "rpca_unrolled_adjoint")
    return np.array(zb[:], dtype=np.float64)


def _f32(t, n=None):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 device tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} values")
    return _ptr(t)


def rpca_mlp_forward(theta, phi, o=None, stream=None):
    """o[b] = network(phi[b]); phi: (B, 4) float32 device."""
    B = phi.shape[0]
    if o is None:
        o = torch.empty((B,), dtype=torch.float32, device=phi.device)
    _check(_lib().rpca_mlp_forward(_f32(theta, RPCA_MLP_PARAMS), _f32(phi, 4 * B), B, _f32(o, B), _stream(stream)),
           "rpca_mlp_forward")
    return o


def rpca_mlp_backward(theta, phi, grad_o, grad=None, stream=None):
    B = phi.shape[0]
    if grad is None:
        grad = torch.empty((RPCA_MLP_PARAMS,), dtype=torch.float32, device=phi.device)
    _check(_lib().rpca_mlp_backward(_f32(theta, RPCA_MLP_PARAMS), _f32(phi, 4 * B), _f32(grad_o, B), B,
                                    _f32(grad, RPCA_MLP_PARAMS), _stream(stream)), "rpca_mlp_backward")
    return grad


def rpca_mlp_adam(theta, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_lib().rpca_mlp_adam(_f32(theta, RPCA_MLP_PARAMS), _f32(m, RPCA_MLP_PARAMS), _f32(v, RPCA_MLP_PARAMS),
                                _f32(grad, RPCA_MLP_PARAMS), int(t), float(lr), float(beta1), float(beta2),
                                float(eps), _stream(stream)), "rpca_mlp_adam")


def rpca_solve(D, params, state, err_hist, zeta_hist, ws, stream=None) -> int:
    """err_hist / zeta_hist: ctypes double arrays (or None)."""
    w, nb = _ws(ws)
    cap = 0 if err_hist is None else len(err_hist)
    return _check(_lib().rpca_solve(_ptr(D), ctypes.byref(params), ctypes.byref(state), err_hist, zeta_hist,
                                    cap, w, nb, _stream(stream)), "rpca_solve")


RPCA_MANY_MAX_STREAMS = 16


def rpca_solve_many(Ds, params, states, err_hists, zeta_hists, wss, streams) -> list:
    """Runs len(Ds) solves together (rpca_solve_many): instance i on
    streams[i % len(streams)] (torch streams). err_hists / zeta_hists: lists of
    ctypes double arrays of one length, or None. Returns the per-instance
    statuses; raises on a negative one."""
    n = len(Ds)
    vp = ctypes.c_void_p
    d_arr = (vp * n)(*[D.data_ptr() for D in Ds])
    p_arr = (ctypes.POINTER(Params) * n)(*[ctypes.pointer(p) for p in params])
    s_arr = (ctypes.POINTER(State) * n)(*[ctypes.pointer(s) for s in states])
    pd = ctypes.POINTER(ctypes.c_double)
    cap = 0 if err_hists is None else len(err_hists[0])
    eh = (pd * n)(*[ctypes.cast(h, pd) for h in err_hists]) if err_hists is not None else None
    zh = (pd * n)(*[ctypes.cast(h, pd) for h in zeta_hists]) if zeta_hists is not None else None
    w_arr = (vp * n)(*[w.data_ptr() for w in wss])
    b_arr = (ctypes.c_size_t * n)(*[w.numel() * w.element_size() for w in wss])
    st_arr = (vp * len(streams))(*[s.cuda_stream for s in streams])
    status = (ctypes.c_int32 * max(n, 1))()
    rc = _lib().rpca_solve_many(n, d_arr, p_arr, s_arr, eh, zh, cap, w_arr, b_arr, st_arr, len(streams), status)
    out = list(status[:n])
    _check(rc, "rpca_solve_many")
    return out


def rpca_materialize(D, params, state, L_out, S_out, ws, stream=None) -> int:
    w, nb = _ws(ws)
    ldl = 0 if L_out is None else L_out.stride(0)
    lds = 0 if S_out is None else S_out.stride(0)
    return _check(_lib().rpca_materialize(_ptr(D), ctypes.byref(params), ctypes.byref(state), _ptr(L_out), ldl,
                                          _ptr(S_out), lds, w, nb, _stream(stream)), "rpca_materialize")


def rpca_tangent_products(D, params, A_L, B_L, zeta, U_t, V_t, Y1, Y2, ws, stream=None) -> float:
    w, nb = _ws(ws)
    out = ctypes.c_double(0.0)
    _check(_lib().rpca_tangent_products(_ptr(D), ctypes.byref(params), _ptr(A_L), _ptr(B_L), float(zeta),
                                        _ptr(U_t), _ptr(V_t), _ptr(Y1), _ptr(Y2), ctypes.byref(out), w, nb,
                                        _stream(stream)), "rpca_tangent_products")
    return float(out.value)


RPCA_PROBE_SINK = 8192


def rpca_read_probe(data: torch.Tensor, sink: torch.Tensor, stream=None) -> None:
    """One read of every byte of `data` (a contiguous device tensor) with no
    arithmetic: the bandwidth reference of the streaming pass."""
    if not data.is_contiguous() or sink.dtype != torch.float32 or sink.numel() < RPCA_PROBE_SINK:
        raise ValueError("contiguous data and a float32 sink of RPCA_PROBE_SINK values are required")
    nbytes = data.numel() * data.element_size()
    _check(_lib().rpca_read_probe(_ptr(data), nbytes - nbytes % 16, _ptr(sink), _stream(stream)),
           "rpca_read_probe")


def rpca_profile_enable(on: bool) -> None:
    _check(_lib().rpca_profile_enable(1 if on else 0), "rpca_profile_enable")


def rpca_profile_read(kind: int | None = None):
    """Per kind of streaming pass ([0] loop, dtype of D; [1] loop, BF16 product;
    [2] initialisation): summed milliseconds and pass counts since the last
    read. With kind given, that kind's (ms, count); otherwise the totals."""
    ms = (ctypes.c_double * RPCA_PROF_KINDS)()
    n = (ctypes.c_int64 * RPCA_PROF_KINDS)()
    _check(_lib().rpca_profile_read(ms, n), "rpca_profile_read")
    if kind is None:
        return float(sum(ms)), int(sum(n))
    return float(ms[kind]), int(n[kind])


def rpca_profile_read_all():
    """[(ms, count)] of the loop's dtype passes, its BF16-product passes, the
    initialisation's passes and whole loop bodies."""
    ms = (ctypes.c_double * RPCA_PROF_KINDS)()
    n = (ctypes.c_int64 * RPCA_PROF_KINDS)()
    _check(_lib().rpca_profile_read(ms, n), "rpca_profile_read")
    return [(float(ms[k]), int(n[k])) for k in range(RPCA_PROF_KINDS)]


# ---- convenience wrapper -----------------------------------------------------

@dataclasses.dataclass
class SolveInfo:
    status: int
    iterations: int
    err: float
    zeta: float
    err_hist: list
    zeta_hist: list
    init_passes: int
    svd_sweeps: int


def make_params(D: torch.Tensor, r: int, beta: float, beta_init: float, gamma: float, mu: float,
                tol: float = 1e-5, max_iter: int = 100, trim: bool = True, init_block: int = 0,
                init_max_passes: int = 0, seed: int = 0, mixed: bool = False, mixed_err: float = 0.0,
                training: bool = False, learned: torch.Tensor | None = None) -> Params:
    if D.dim() != 2 or D.stride(1) != 1:
        raise ValueError("D must be a 2-D row-major tensor with unit column stride")
    if D.dtype == torch.float64:
        dt = RPCA_F64
    elif D.dtype == torch.float32:
        dt = RPCA_F32
    else:
        raise ValueError("D must be float32 or float64")
    return Params(m=D.shape[0], n=D.shape[1], ldd=D.stride(0), r=int(r), dtype=dt, beta=float(beta),
                  beta_init=float(beta_init), gamma=float(gamma), mu=float(mu) if trim else 0.0, tol=float(tol),
                  max_iter=int(max_iter), init_block=int(init_block), init_max_passes=int(init_max_passes),
                  flags=((0 if trim else RPCA_FLAG_NO_TRIM) | (RPCA_FLAG_MIXED if mixed else 0)
                         | (RPCA_FLAG_TRAINING if training else 0) | (RPCA_FLAG_LEARNED if learned is not None else 0)),
                  seed=int(seed), mixed_err=float(mixed_err),
                  zeta_mlp=(_f32(learned, RPCA_MLP_PARAMS) if learned is not None else None))


RPCA_BATCH_MAX = 65535


class BatchSolver:
    """Many instances of one shape solved together (rpca_solve_batch): every
    kernel launch covers all of them. Owns one device slab per instance
    (its D, its iterate and its workspace, rpca_batch_layout_of)."""

    def __init__(self, D: torch.Tensor, r: int, beta, beta_init, gamma, mu, tol=1e-5, max_iter: int = 100,
                 trim: bool = True, init_block: int = 0, init_max_passes: int = 0, seed: int = 0,
                 mixed: bool = False, learned: torch.Tensor | None = None):
        """D: (count, m, n) device tensor (float32 or float64); copied into the
        slabs. beta, beta_init, gamma, mu, tol: one value for all instances or
        one per instance."""
        if not D.is_cuda or D.dim() != 3:
            raise ValueError("D must be a (count, m, n) device tensor")
        count, m, n = D.shape
        if not 1 <= count <= RPCA_BATCH_MAX:
            raise ValueError("1 <= count <= RPCA_BATCH_MAX")
        self.count = count

        def each(v):
            v = list(v) if isinstance(v, (list, tuple, np.ndarray)) else [v] * count
            if len(v) != count:
                raise ValueError("one value or one per instance")
            return [float(x) for x in v]

        b, bi, g, mu_, tl = each(beta), each(beta_init), each(gamma), each(mu), each(tol)
        self.params_all = (Params * count)()
        for i in range(count):
            self.params_all[i] = make_params(D[0], r, b[i], bi[i], g[i], mu_[i], tl[i], max_iter, trim, init_block,
                                             init_max_passes, seed, mixed, 0.0, False, learned)
            self.params_all[i].ldd = n
        self.params = self.params_all[0]
        self._learned = learned
        lay = BatchLayout()
        _check(_lib().rpca_batch_layout_of(ctypes.byref(self.params), ctypes.byref(lay)), "rpca_batch_layout_of")
        self.layout = lay
        sb = lay.slab_bytes
        raw = torch.empty(count * sb + 256, dtype=torch.uint8, device=D.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.slabs = raw[off:off + count * sb].view(count, sb)
        esz = D.element_size()

        def region(o, nbytes, dtype, shape):
            return self.slabs[:, o:o + nbytes].view(dtype).view((count,) + shape)

        self.D = region(lay.off_D, m * n * esz, D.dtype, (m, n))
        self.U = region(lay.off_U, m * r * 8, torch.float64, (m, r))
        self.V = region(lay.off_V, n * r * 8, torch.float64, (n, r))
        self.sigma = region(lay.off_sigma, r * 8, torch.float64, (r,))
        self.D.copy_(D)

    def solve(self):
        """Solves every instance; returns their SolveInfo (status per instance)."""
        n = self.count
        cap = self.params.max_iter + 1
        eh = (ctypes.c_double * (n * cap))()
        zh = (ctypes.c_double * (n * cap))()
        st = (State * n)()
        status = (ctypes.c_int32 * n)()
        torch.cuda.current_stream(self.D.device).synchronize()
        rc = _lib().rpca_solve_batch(n, ctypes.c_void_p(self.slabs.data_ptr()), self.params_all, st,
                                     eh, zh, cap, status, _stream(None))
        if rc < 0 and all(s >= 0 for s in status[:n]):
            _check(rc, "rpca_solve_batch")
        out = []
        for i in range(n):
            k = st[i].k
            out.append(SolveInfo(status=status[i], iterations=k, err=st[i].err, zeta=st[i].zeta,
                                 err_hist=list(eh[i * cap:i * cap + k + 1]), zeta_hist=list(zh[i * cap:i * cap + k + 1]),
                                 init_passes=st[i].init_passes, svd_sweeps=st[i].svd_sweeps))
        return out


class Solver:
    """Owns the iterate buffers (U, sigma, V in FP64) and the workspace for one D."""

    def __init__(self, D: torch.Tensor, r: int, beta: float, beta_init: float, gamma: float, mu: float,
                 tol: float = 1e-5, max_iter: int = 100, trim: bool = True, init_block: int = 0,
                 init_max_passes: int = 0, seed: int = 0, mixed: bool = False, mixed_err: float = 0.0,
                 training: bool = False, learned: torch.Tensor | None = None):
        if not D.is_cuda:
            raise ValueError("D must be a device tensor")
        self.D = D
        self.params = make_params(D, r, beta, beta_init, gamma, mu, tol, max_iter, trim, init_block,
                                  init_max_passes, seed, mixed, mixed_err, training, learned)
        self._learned = learned   # keeps the parameters alive while the params point at them
        dev = D.device
        m, n = D.shape
        self.U = torch.zeros((m, r), dtype=torch.float64, device=dev)
        self.V = torch.zeros((n, r), dtype=torch.float64, device=dev)
        self.sigma = torch.zeros((r,), dtype=torch.float64, device=dev)
        nbytes = rpca_workspace_size(self.params)
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws = raw[off:off + nbytes]
        self.state = State(U=self.U.data_ptr(), V=self.V.data_ptr(), sigma=self.sigma.data_ptr(),
                           zeta=0.0, err=float("nan"), sigma1_pt=0.0, sigma_r1_pt=0.0, normD=0.0, k=0,
                           init_passes=0)

    # state as host values / tensors
    def set_state(self, U, sigma, V, zeta: float, k: int, normD: float = 0.0):
        def host(a):
            return a if isinstance(a, torch.Tensor) else torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)
        self.U.copy_(host(U))
        self.V.copy_(host(V))
        self.sigma.copy_(host(sigma))
        self.state.zeta = float(zeta)
        self.state.k = int(k)
        self.state.normD = float(normD)
        self.state.err = float("nan")

    def init(self) -> None:
        rpca_init(self.D, self.params, self.state, self.ws)

    def step(self) -> None:
        rpca_step(self.D, self.params, self.state, self.ws)

    def step_noalloc(self) -> None:
        rpca_step_noalloc(self.D, self.params, self.state)

    def trim(self):
        m, n = self.D.shape
        r = self.params.r
        Ut = torch.empty((m, r), dtype=torch.float64, device=self.D.device)
        Vt = torch.empty((n, r), dtype=torch.float64, device=self.D.device)
        rpca_trim(self.params, self.state, Ut, Vt, self.ws)
        return Ut, Vt

    def solve(self) -> SolveInfo:
        cap = self.params.max_iter + 1
        eh = (ctypes.c_double * cap)()
        zh = (ctypes.c_double * cap)()
        st = rpca_solve(self.D, self.params, self.state, eh, zh, self.ws)
        k = self.state.k
        return SolveInfo(status=st, iterations=k, err=self.state.err, zeta=self.state.zeta,
                         err_hist=list(eh[:k + 1]), zeta_hist=list(zh[:k + 1]),
                         init_passes=self.state.init_passes, svd_sweeps=self.state.svd_sweeps)

    def materialize(self, want_L: bool = True, want_S: bool = True):
        L = torch.empty_like(self.D) if want_L else None
        S = torch.empty_like(self.D) if want_S else None
        rpca_materialize(self.D, self.params, self.state, L, S, self.ws)
        return L, S

    def tangent_products(self, A_L, B_L, zeta, U_t, V_t):
        m, n = self.D.shape
        r = self.params.r
        Y1 = torch.empty((m, r), dtype=torch.float64, device=self.D.device)
        Y2 = torch.empty((n, r), dtype=torch.float64, device=self.D.device)
        res = rpca_tangent_products(self.D, self.params, A_L.contiguous(), B_L.contiguous(), zeta,
                                    U_t.contiguous(), V_t.contiguous(), Y1, Y2, self.ws)
        return Y1, Y2, res

    def L_factors(self):
        return self.U, self.sigma, self.V

    def relaxed_step(self, zeta: float, tau: float, P: torch.Tensor, Q: torch.Tensor) -> RelaxResult:
        """One relaxed iteration from the current state (needs training=True)."""
        return rpca_relaxed_step(self.D, self.params, self.state, zeta, tau, P, Q, self.ws)

    def unrolled(self, zetas, taus, weights, P: torch.Tensor, Q: torch.Tensor):
        """K relaxed iterations from the current state (which advances to L_K),
        keeping the factor checkpoints. Returns (losses, checkpoints)."""
        ck = [(self.U.clone(), self.sigma.clone(), self.V.clone())]
        losses = []
        for z, t in zip(zetas, taus):
            res = self.relaxed_step(float(z), float(t), P, Q)
            losses.append(res.loss)
            ck.append((self.U.clone(), self.sigma.clone(), self.V.clone()))
        return losses, ck

    def unrolled_adjoint(self, checkpoints, zetas, taus, weights, P: torch.Tensor, Q: torch.Tensor):
        """Gradients of sum_k weights[k-1] loss_k over the iterations that
        produced `checkpoints`: (d/dzeta (K values), dU_0, dsigma_0, dV_0)."""
        U0, s0, V0 = checkpoints[0]
        Ub, sb, Vb = torch.empty_like(U0), torch.empty_like(s0), torch.empty_like(V0)
        zb = rpca_unrolled_adjoint(self.D, self.params, [c[0] for c in checkpoints], [c[1] for c in checkpoints],
                                   [c[2] for c in checkpoints], zetas, taus, weights, P, Q, Ub, sb, Vb, self.ws)
        return zb, Ub, sb, Vb

    def get_state(self):
        """(U, sigma, V, zeta, k, normD) copies of the current state."""
        return (self.U.clone(), self.sigma.clone(), self.V.clone(), self.state.zeta, self.state.k,
                self.state.normD)

    def put_state(self, saved) -> None:
        U, s, V, zeta, k, normD = saved
        self.U.copy_(U)
        self.sigma.copy_(s)
        self.V.copy_(V)
        self.state.zeta, self.state.k, self.state.normD = float(zeta), int(k), float(normD)


def solve_many(solvers, n_streams: int = 8) -> list:
    """Solves the problems of several Solver objects together
    (rpca_solve_many) on n_streams new streams; returns their SolveInfo."""
    n_streams = max(1, min(n_streams, RPCA_MANY_MAX_STREAMS, len(solvers)))
    dev = solvers[0].D.device if solvers else torch.device("cuda")
    streams = [torch.cuda.Stream(device=dev) for _ in range(n_streams)]
    cap = max(sv.params.max_iter for sv in solvers) + 1 if solvers else 1
    eh = [(ctypes.c_double * cap)() for _ in solvers]
    zh = [(ctypes.c_double * cap)() for _ in solvers]
    torch.cuda.current_stream(dev).synchronize()   # inputs written on the current stream are complete
    status = rpca_solve_many([sv.D for sv in solvers], [sv.params for sv in solvers], [sv.state for sv in solvers],
                             eh, zh, [sv.ws for sv in solvers], streams)
    out = []
    for sv, st, e, z in zip(solvers, status, eh, zh):
        k = sv.state.k
        out.append(SolveInfo(status=st, iterations=k, err=sv.state.err, zeta=sv.state.zeta, err_hist=list(e[:k + 1]),
                             zeta_hist=list(z[:k + 1]), init_passes=sv.state.init_passes,
                             svd_sweeps=sv.state.svd_sweeps))
    return out


RPCA_BATCH_BUFS = 4   # batched calls that run on one device at once


def solve_batches(batches, n_streams: int = 3) -> list:
    """Solves several BatchSolver objects (batches of different shapes or
    ranks) concurrently: n_streams host threads, each on its own new stream,
    take the batches in order of decreasing size (instances x m x n x r), each
    thread the batch that keeps its queue shortest. One batch's streaming pass
    then overlaps the latency-bound kernels of another. Returns each batch's
    list of SolveInfo, in the order of `batches`; results are those of
    solving the batches one after another. All batches are on one device."""
    import threading
    n_streams = max(1, min(n_streams, RPCA_BATCH_BUFS, len(batches)))
    if not batches:
        return []
    dev = batches[0].D.device
    if any(bs.D.device != dev for bs in batches):
        raise ValueError("solve_batches: every batch must be on one device")
    torch.cuda.current_stream(dev).synchronize()   # slabs written on the current stream are complete
    cost = [bs.count * bs.params.m * bs.params.n * bs.params.r for bs in batches]
    queues, load = [[] for _ in range(n_streams)], [0] * n_streams
    for i in sorted(range(len(batches)), key=lambda i: -cost[i]):
        q = min(range(n_streams), key=lambda k: load[k])
        queues[q].append(i)
        load[q] += cost[i]
    streams = [torch.cuda.Stream(device=dev) for _ in range(n_streams)]
    out, errors = [None] * len(batches), []

    def work(k):
        try:
            with torch.cuda.device(dev), torch.cuda.stream(streams[k]):
                for i in queues[k]:
                    out[i] = batches[i].solve()
        except BaseException as e:   # re-raised in the calling thread
            errors.append(e)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(n_streams)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    if errors:
        raise errors[0]
    return out


class UnrolledRelaxed(torch.autograd.Function):
    """loss = UnrolledRelaxed.apply(zetas, U0, sigma0, V0, solver, P, Q, taus, weights):
    K = len(zetas) relaxed iterations of `solver` from L_0 = U0 diag(sigma0) V0^T
    (the solver's state ends at L_K) and the weighted loss
    sum_k weights[k-1] ||L_k - P Q^T||^2 / ||P Q^T||^2. Backward runs the
    library's reverse sweep over the iterations from the factor checkpoints:
    gradients for the thresholds and for the initial factors."""

    @staticmethod
    def forward(ctx, zetas, U0, sigma0, V0, solver, P, Q, taus, weights):
        z = [float(v) for v in zetas.detach().cpu()]
        solver.U.copy_(U0.detach())
        solver.sigma.copy_(sigma0.detach())
        solver.V.copy_(V0.detach())
        losses, ck = solver.unrolled(z, taus, weights, P, Q)
        ctx.solver, ctx.ck, ctx.z = solver, ck, z
        ctx.taus, ctx.weights, ctx.P, ctx.Q = list(taus), list(weights), P, Q
        ctx.losses = losses
        return torch.tensor(sum(w * l for w, l in zip(weights, losses)), dtype=torch.float64, device=zetas.device)

    @staticmethod
    def backward(ctx, grad_loss):
        zb, Ub, sb, Vb = ctx.solver.unrolled_adjoint(ctx.ck, ctx.z, ctx.taus, ctx.weights, ctx.P, ctx.Q)
        g = grad_loss.to(torch.float64)
        gz = torch.as_tensor(zb, dtype=torch.float64, device=grad_loss.device) * g
        return gz, Ub * g, sb * g, Vb * g, None, None, None, None, None


class RelaxedStep(torch.autograd.Function):
    """loss = RelaxedStep.apply(zeta, solver, P, Q, tau): one relaxed iteration
    of `solver` (its state advances to L_{k+1}) with the hand-written adjoint
    in zeta. The state is data here, not a differentiable input: backward
    returns d loss / d zeta (times the incoming gradient) and nothing else."""

    @staticmethod
    def forward(ctx, zeta, solver, P, Q, tau):
        res = solver.relaxed_step(float(zeta), float(tau), P, Q)
        ctx.dloss = res.dloss_dzeta
        ctx.result = res
        return torch.tensor(res.loss, dtype=torch.float64, device=zeta.device)

    @staticmethod
    def backward(ctx, grad_loss):
        g = grad_loss * ctx.dloss
        return g, None, None, None, None
