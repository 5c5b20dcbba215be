"""parapn: parallel-in-time probabilistic numerical ODE solver (ParaIEKS) on MI355X.

Thin Python binding over the C ABI of ``libparapn.so`` (include/parapn.h).
It only marshals arguments: PyTorch provides device memory and the current
HIP stream; every step of the solver runs in the library's HIP kernels.
There is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libparapn.so")

OK, MAXITER, EINVAL, ENOMEM, EDEVICE, ENONFINITE = 0, 1, -1, -2, -3, -4
FP64, FP32_SQRT = 0, 1

FIELDS = {
    "logistic": 0,
    "fhn": 1,
    "lorenz": 2,
    "lotka_volterra": 3,
    "mol_heat_reaction": 4,
    "affine": 5,
    "rigid_body": 6,
    "van_der_pol": 7,
}
FIELD_DIM = {"logistic": 1, "fhn": 2, "lorenz": 3, "lotka_volterra": 2, "rigid_body": 3, "van_der_pol": 2}
PRECISIONS = {"fp64": FP64, "fp32": FP32_SQRT, "fp32_sqrt": FP32_SQRT}
PRIORS = {"iwp": 0, "ioup": 1, "matern": 2}
INITS = {"constant": 0, "coarse": 1}
STARTS = {0: "constant", 1: "coarse", 2: "given", 3: "coarse_failed"}
STOP_RULES = {"trajectory": 1, "objective": 2, "either": 3}
LINEARIZATIONS = {"ek1": 0, "ek0": 1, "diag_ek1": 2}
EXPORTED = ["parapn_create", "parapn_destroy", "parapn_workspace_size", "parapn_solve", "parapn_solve_batch",
            "parapn_start_trajectory", "parapn_pararts_noalloc",
            "parapn_pararts", "parapn_pararts_tv",
            "parapn_filter_combine", "parapn_profile_enable", "parapn_profile_only", "parapn_profile_read",
            "parapn_server_create", "parapn_server_destroy", "parapn_server_clock", "parapn_server_submit", "parapn_server_step",
            "parapn_server_poll", "parapn_server_footprint", "parapn_server_stats", "parapn_last_error"]


class ParapnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("parapn error %d: %s" % (code, msg))
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [
        ("field", ctypes.c_int32),
        ("d", ctypes.c_int32),
        ("params", ctypes.POINTER(ctypes.c_double)),
        ("n_params", ctypes.c_int32),
        ("y0", ctypes.POINTER(ctypes.c_double)),
        ("t0", ctypes.c_double),
        ("t1", ctypes.c_double),
        ("q", ctypes.c_int32),
        ("N", ctypes.c_int64),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("fixed_iters", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("init_traj", ctypes.POINTER(ctypes.c_double)),
        ("init_on_device", ctypes.c_int32),
        ("lm_sigma", ctypes.c_double),
        ("prior", ctypes.c_int32),
        ("prior_theta", ctypes.c_double),
        ("init_mode", ctypes.c_int32),
        ("coarse_points", ctypes.c_int32),
        ("stop_rule", ctypes.c_int32),
        ("obj_atol", ctypes.c_double),
        ("obj_rtol", ctypes.c_double),
        ("calibrate", ctypes.c_int32),
        ("linearization", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("final_delta", ctypes.c_double),
        ("tol_used", ctypes.c_double),
        ("delta_history", ctypes.POINTER(ctypes.c_double)),
        ("start", ctypes.c_int32),
        ("sigma_hat", ctypes.c_double),
        ("objective", ctypes.c_double),
        ("objective_history", ctypes.POINTER(ctypes.c_double)),
    ]


class Completion(ctypes.Structure):
    _fields_ = [
        ("req_id", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("final_delta", ctypes.c_double),
        ("t_submit", ctypes.c_double),
        ("t_start", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("start", ctypes.c_int32),
        ("sigma_hat", ctypes.c_double),
        ("objective", ctypes.c_double),
    ]


_lib = None
_ctx = {}


def load_library(path: str = LIB_PATH):
    """Load libparapn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libparapn.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2310_01145_amd.build)")
    L = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.parapn_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, sz]
    L.parapn_create.restype = ctypes.c_int
    L.parapn_destroy.argtypes = [vp]
    L.parapn_destroy.restype = None
    L.parapn_workspace_size.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(sz)]
    L.parapn_workspace_size.restype = ctypes.c_int
    L.parapn_solve.argtypes = [vp, ctypes.POINTER(Problem), vp, vp, ctypes.POINTER(Info), vp]
    L.parapn_solve.restype = ctypes.c_int
    L.parapn_start_trajectory.argtypes = [vp, ctypes.POINTER(Problem), vp, ctypes.POINTER(i32), vp]
    L.parapn_start_trajectory.restype = ctypes.c_int
    L.parapn_solve_batch.argtypes = [vp, ctypes.POINTER(Problem), i32, ctypes.POINTER(ctypes.c_double), vp, vp,
                                      ctypes.POINTER(Info), vp]
    L.parapn_solve_batch.restype = ctypes.c_int
    L.parapn_pararts.argtypes = [vp, i32, i32, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.parapn_pararts.restype = ctypes.c_int
    L.parapn_pararts_tv.argtypes = [vp, i32, i32, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.parapn_pararts_tv.restype = ctypes.c_int
    L.parapn_filter_combine.argtypes = [vp, i32, i64, i32, vp, vp, vp, vp]
    L.parapn_filter_combine.restype = ctypes.c_int
    L.parapn_profile_enable.argtypes = [ctypes.c_int]
    L.parapn_profile_enable.restype = ctypes.c_int
    L.parapn_profile_only.argtypes = [ctypes.c_char_p]
    L.parapn_profile_only.restype = ctypes.c_int
    L.parapn_profile_read.argtypes = [i32, ctypes.c_char_p, i32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32)]
    L.parapn_profile_read.restype = ctypes.c_int
    L.parapn_server_create.argtypes = [ctypes.POINTER(vp), vp, i32, sz, vp]
    L.parapn_server_create.restype = ctypes.c_int
    L.parapn_server_destroy.argtypes = [vp]
    L.parapn_server_destroy.restype = None
    L.parapn_server_clock.argtypes = []
    L.parapn_server_clock.restype = ctypes.c_double
    L.parapn_server_submit.argtypes = [vp, ctypes.POINTER(Problem), ctypes.c_uint64, vp, vp]
    L.parapn_server_submit.restype = ctypes.c_int
    L.parapn_server_step.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.parapn_server_step.restype = ctypes.c_int
    L.parapn_server_poll.argtypes = [vp, ctypes.POINTER(Completion), i32, ctypes.POINTER(i32)]
    L.parapn_server_poll.restype = ctypes.c_int
    L.parapn_server_footprint.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(sz)]
    L.parapn_server_footprint.restype = ctypes.c_int
    L.parapn_server_stats.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64)]
    L.parapn_server_stats.restype = ctypes.c_int
    L.parapn_last_error.argtypes = []
    L.parapn_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def last_error() -> str:
    return load_library().parapn_last_error().decode()


def _check(rc, allow=(OK,)):
    if rc not in allow:
        raise ParapnError(rc, last_error())
    return rc


def context(device: int = 0, budget: int = 0):
    key = (device, budget)
    if key not in _ctx:
        L = load_library()
        h = ctypes.c_void_p()
        _check(L.parapn_create(ctypes.byref(h), device, budget))
        _ctx[key] = h
    return _ctx[key]


def _torch():
    import torch

    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dtype(precision):
    torch = _torch()
    return torch.float64 if precision == FP64 else torch.float32


def make_problem(field, params, y0, t0, t1, q, N, *, precision="fp64", tol=1e-10, max_iter=20, fixed_iters=0,
                 init_traj=None, d=None, lm_sigma=0.0, prior="iwp", theta=0.0, init="constant", coarse_points=0,
                 stop_rule="trajectory", obj_atol=1e-9, obj_rtol=1e-6, calibrate=False, linearization="ek1"):
    """Build the ctypes Problem (keeps the host arrays alive on the object)."""
    fid = FIELDS[field] if isinstance(field, str) else int(field)
    y0 = np.ascontiguousarray(np.asarray(y0, dtype=np.float64).ravel())
    prm = np.ascontiguousarray(np.asarray(params if params is not None else [], dtype=np.float64).ravel())
    pb = Problem()
    pb.field = fid
    pb.d = int(d if d is not None else y0.size)
    pb.params = prm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if prm.size else None
    pb.n_params = prm.size
    pb.y0 = y0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    pb.t0, pb.t1 = float(t0), float(t1)
    pb.q = int(q)
    pb.N = int(N)
    pb.tol = float(tol)
    pb.max_iter = int(max_iter)
    pb.fixed_iters = int(fixed_iters)
    pb.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    pb.lm_sigma = float(lm_sigma)
    pb.prior = PRIORS[prior] if isinstance(prior, str) else int(prior)
    pb.prior_theta = float(theta)
    pb.init_mode = INITS[init] if isinstance(init, str) else int(init)
    pb.coarse_points = int(coarse_points)
    pb.stop_rule = STOP_RULES[stop_rule] if isinstance(stop_rule, str) else int(stop_rule)
    pb.obj_atol = float(obj_atol)
    pb.obj_rtol = float(obj_rtol)
    pb.calibrate = 1 if calibrate else 0
    pb.linearization = LINEARIZATIONS[linearization] if isinstance(linearization, str) else int(linearization)
    keep = [y0, prm]
    pb.init_on_device = 0
    if init_traj is not None and hasattr(init_traj, "is_cuda") and init_traj.is_cuda:
        # a device tensor [N+1, D] of float64, read on the solve's stream
        D = pb.d * (pb.q + 1)
        if init_traj.dtype != _torch().float64 or tuple(init_traj.shape) != (pb.N + 1, D) \
                or not init_traj.is_contiguous():
            raise ValueError("device init_traj must be a contiguous float64 tensor of shape (N+1, D)")
        pb.init_traj = ctypes.cast(ctypes.c_void_p(init_traj.data_ptr()), ctypes.POINTER(ctypes.c_double))
        pb.init_on_device = 1
        keep.append(init_traj)
    elif init_traj is not None:
        it = np.ascontiguousarray(np.asarray(init_traj, dtype=np.float64))
        pb.init_traj = it.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        keep.append(it)
    else:
        pb.init_traj = None
    pb._keep = keep
    return pb


def workspace_size(problem: Problem) -> int:
    n = ctypes.c_size_t()
    _check(load_library().parapn_workspace_size(ctypes.byref(problem), ctypes.byref(n)))
    return n.value


def solve(field, params, y0, t0, t1, q, N, *, precision="fp64", tol=1e-10, max_iter=20, fixed_iters=0,
          init_traj=None, want_cov=False, device=0, stream=None, out=None, d=None, lm_sigma=0.0, prior="iwp",
          theta=0.0, init="constant", coarse_points=0, stop_rule="trajectory", obj_atol=1e-9, obj_rtol=1e-6,
          calibrate=False, linearization="ek1"):
    """ParaIEKS (Alg. 2) on the GPU.  Returns a dict with ``mean`` [N+1, D]
    (original coordinates, torch tensor on the device), ``sqrtcov``
    [N+1, D, D] or None, ``status``, ``iterations``, ``deltas``,
    ``converged``, ``tol_used``, ``start``, ``sigma_hat`` (quasi-MLE
    diffusion), ``objective`` and ``objectives`` (V after each iteration).
    ``stop_rule``: "trajectory", "objective" or "either" (Sec. 3.2.2);
    ``calibrate`` scales the returned factors by sigma_hat.  ``lm_sigma`` > 0 damps each
    Gauss-Newton step (Levenberg-Marquardt, see parapn_problem.lm_sigma);
    ``init="coarse"`` starts from the coarse-grid smoother
    (parapn_problem.init_mode) with ``coarse_points`` coarse steps (0: the
    library's default).  ``linearization``: "ek1", "ek0" or "diag_ek1"
    (parapn_problem.linearization)."""
    torch = _torch()
    L = load_library()
    pb = make_problem(field, params, y0, t0, t1, q, N, precision=precision, tol=tol, max_iter=max_iter,
                      fixed_iters=fixed_iters, init_traj=init_traj, d=d, lm_sigma=lm_sigma, prior=prior, theta=theta,
                      init=init, coarse_points=coarse_points, stop_rule=stop_rule, obj_atol=obj_atol,
                      obj_rtol=obj_rtol, calibrate=calibrate, linearization=linearization)
    D = pb.d * (pb.q + 1)
    dt = _dtype(pb.precision)
    dev = torch.device("cuda", device)
    if out is not None:
        mean, cov = out
    else:
        mean = torch.empty((pb.N + 1, D), dtype=dt, device=dev)
        cov = torch.empty((pb.N + 1, D, D), dtype=dt, device=dev) if want_cov else None
    hist = np.zeros(max(pb.max_iter, pb.fixed_iters, 1))
    ohist = np.zeros_like(hist)
    info = Info()
    info.delta_history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    info.objective_history = ohist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rc = L.parapn_solve(context(device), ctypes.byref(pb), _dptr(mean), _dptr(cov), ctypes.byref(info),
                        _stream_handle(stream))
    _check(rc, allow=(OK, MAXITER, ENONFINITE))
    k = info.iterations
    return {"mean": mean, "sqrtcov": cov, "status": rc, "iterations": k, "deltas": hist[:k].copy(),
            "converged": bool(info.converged), "tol_used": info.tol_used, "final_delta": info.final_delta,
            "start": STARTS.get(info.start, info.start), "sigma_hat": info.sigma_hat, "objective": info.objective,
            "objectives": ohist[:k].copy()}


def start_trajectory(field, params, y0, t0, t1, q, N, *, precision="fp64", init="coarse", coarse_points=0,
                     init_traj=None, d=None, device=0, stream=None):
    """The starting trajectory a solve would use: (float64 device tensor
    [N+1, D] in original coordinates, start name)."""
    torch = _torch()
    L = load_library()
    pb = make_problem(field, params, y0, t0, t1, q, N, precision=precision, init_traj=init_traj, d=d, init=init,
                      coarse_points=coarse_points)
    D = pb.d * (pb.q + 1)
    out = torch.empty((pb.N + 1, D), dtype=torch.float64, device=torch.device("cuda", device))
    st = ctypes.c_int32()
    _check(L.parapn_start_trajectory(context(device), ctypes.byref(pb), _dptr(out), ctypes.byref(st),
                                     _stream_handle(stream)))
    return out, STARTS.get(st.value, st.value)


def solve_batch(field, params, y0s, t0, t1, q, N, *, precision="fp64", tol=1e-10, max_iter=20, fixed_iters=0,
                want_cov=False, device=0, stream=None, prior="iwp", theta=0.0, linearization="ek1",
                stop_rule="trajectory", obj_atol=1e-9, obj_rtol=1e-6, calibrate=False, init_traj=None):
    """Alg. 2 for a batch of initial values ``y0s`` [B, d] of one problem
    (parapn_solve_batch).  Returns ``mean`` [B, N+1, D], ``sqrtcov``
    [B, N+1, D, D] or None, the overall ``status`` and per-instance
    ``iterations``, ``converged``, ``final_delta``, ``deltas``,
    ``sigma_hat``, ``objective`` and ``objectives``."""
    torch = _torch()
    L = load_library()
    y0s = np.ascontiguousarray(np.asarray(y0s, dtype=np.float64))
    if y0s.ndim != 2:
        raise ValueError("y0s must be [batch, d]")
    B, d = y0s.shape
    pb = make_problem(field, params, y0s[0], t0, t1, q, N, precision=precision, tol=tol, max_iter=max_iter,
                      fixed_iters=fixed_iters, d=d, prior=prior, theta=theta, linearization=linearization,
                      stop_rule=stop_rule, obj_atol=obj_atol, obj_rtol=obj_rtol, calibrate=calibrate,
                      init_traj=init_traj)
    D = d * (pb.q + 1)
    dt = _dtype(pb.precision)
    dev = torch.device("cuda", device)
    mean = torch.empty((B, pb.N + 1, D), dtype=dt, device=dev)
    cov = torch.empty((B, pb.N + 1, D, D), dtype=dt, device=dev) if want_cov else None
    cap = max(pb.max_iter, pb.fixed_iters, 1)
    hist = np.zeros((B, cap))
    ohist = np.zeros((B, cap))
    infos = (Info * B)()
    for b in range(B):
        infos[b].delta_history = hist[b].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        infos[b].objective_history = ohist[b].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rc = L.parapn_solve_batch(context(device), ctypes.byref(pb), B, y0s.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              _dptr(mean), _dptr(cov), infos, _stream_handle(stream))
    _check(rc, allow=(OK, MAXITER, ENONFINITE))
    its = [infos[b].iterations for b in range(B)]
    return {"mean": mean, "sqrtcov": cov, "status": rc, "iterations": its,
            "converged": [bool(infos[b].converged) for b in range(B)],
            "final_delta": [infos[b].final_delta for b in range(B)],
            "deltas": [hist[b, :its[b]].copy() for b in range(B)],
            "sigma_hat": [infos[b].sigma_hat for b in range(B)],
            "objective": [infos[b].objective for b in range(B)],
            "objectives": [ohist[b, :its[b]].copy() for b in range(B)]}


def pararts(mu0, sqrt_sigma0, Phi, sqrtQ, H, dvec, *, precision="fp64", want_cov=True, want_filter=True,
            device=0, stream=None):
    """ParaRTS (Alg. 1) on a linear model with noiseless observations
    H_n Y_n = dvec_n.  Inputs are torch tensors on the device with the dtype
    of the precision; H is [N, dobs, D], dvec [N, dobs]; Phi and sqrtQ are
    [D, D] (constant) or [N, D, D] (step n uses entry n-1:
    parapn_pararts_tv)."""
    torch = _torch()
    L = load_library()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    dt = _dtype(prec)
    ins = [x.to(dtype=dt).contiguous() for x in (mu0, sqrt_sigma0, Phi, sqrtQ, H, dvec)]
    N, dobs, D = ins[4].shape
    dev = ins[0].device
    ms = torch.empty((N + 1, D), dtype=dt, device=dev)
    sPs = torch.empty((N + 1, D, D), dtype=dt, device=dev) if want_cov else None
    mf = torch.empty((N + 1, D), dtype=dt, device=dev) if want_filter else None
    sPf = torch.empty((N + 1, D, D), dtype=dt, device=dev) if want_filter else None
    tv = ins[2].dim() == 3
    if tv and (tuple(ins[2].shape) != (N, D, D) or tuple(ins[3].shape) != (N, D, D)):
        raise ValueError("per-step Phi and sqrtQ must be [N, D, D]")
    fn = L.parapn_pararts_tv if tv else L.parapn_pararts
    _check(fn(context(device), D, dobs, N, prec, *[_dptr(x) for x in ins], _dptr(ms), _dptr(sPs), _dptr(mf),
              _dptr(sPf), _stream_handle(stream)))
    return {"mean": ms, "sqrtcov": sPs, "filt_mean": mf, "filt_sqrtcov": sPf}


def filter_combine(a, c, *, precision="fp64", device=0, stream=None):
    """Batched square-root filtering operator: rows of a and c are packed
    elements (A, b, sqrtC, eta, sqrtJ) of 3D^2+2D values each."""
    torch = _torch()
    L = load_library()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    dt = _dtype(prec)
    a = a.to(dtype=dt).contiguous()
    c = c.to(dtype=dt).contiguous()
    count, rec = a.shape
    D = int(round((-2 + (4 + 12 * rec) ** 0.5) / 6))
    assert 3 * D * D + 2 * D == rec, "bad record size"
    out = torch.empty_like(a)
    _check(L.parapn_filter_combine(context(device), D, count, prec, _dptr(a), _dptr(c), _dptr(out),
                                   _stream_handle(stream)))
    return out


def profile_enable(on: bool = True):
    """Start (or stop) per-kernel event timing; clears previous counters."""
    _check(load_library().parapn_profile_enable(1 if on else 0))


def profile_only(kernel=None):
    """Time only launches of this kernel name (None: every kernel)."""
    _check(load_library().parapn_profile_only(kernel.encode() if kernel else None))


def profile_read(max_kernels: int = 64):
    """{kernel name: (total ms, launches)} since profile_enable."""
    L = load_library()
    name_len = 64
    names = ctypes.create_string_buffer(max_kernels * name_len)
    tot = (ctypes.c_double * max_kernels)()
    cnt = (ctypes.c_int64 * max_kernels)()
    n = ctypes.c_int32()
    _check(L.parapn_profile_read(max_kernels, names, name_len, tot, cnt, ctypes.byref(n)))
    out = {}
    for k in range(min(n.value, max_kernels)):
        nm = names.raw[k * name_len:(k + 1) * name_len].split(b"\0", 1)[0].decode()
        out[nm] = (tot[k], cnt[k])
    return out


class Server:
    """Continuous-batching server over the C ABI (parapn_server_*): submit
    IVPs at any time, call ``step()`` to run one Gauss-Newton iteration for
    every admitted request, ``poll()`` for completions.  Output tensors are
    allocated at submission and kept until the completion is polled."""

    def __init__(self, max_slots=64, budget=0, device=0, stream=None, ctx_budget=0):
        """stream: the HIP stream of all the server's work; by default a
        stream of its own (default priority), on which an unchanged pack
        replays a captured graph of its iteration (the legacy default stream
        cannot be captured: on it every launch is issued anew)."""
        torch = _torch()
        self._L = load_library()
        self._device = device
        self._stream = stream if stream is not None else torch.cuda.Stream(device=device)
        h = ctypes.c_void_p()
        _check(self._L.parapn_server_create(ctypes.byref(h), context(device, ctx_budget), int(max_slots), int(budget),
                                            ctypes.c_void_p(self._stream.cuda_stream)))
        self._h = h
        self._pending = {}

    def submit(self, req_id, field, params, y0, t0, t1, q, N, *, precision="fp64", tol=1e-10, max_iter=20,
               fixed_iters=0, d=None, lm_sigma=0.0, prior="iwp", theta=0.0, init="constant", coarse_points=0,
               want_cov=False, stop_rule="trajectory", obj_atol=1e-9, obj_rtol=1e-6, calibrate=False,
               linearization="ek1"):
        torch = _torch()
        pb = make_problem(field, params, y0, t0, t1, q, N, precision=precision, tol=tol, max_iter=max_iter,
                          fixed_iters=fixed_iters, d=d, lm_sigma=lm_sigma, prior=prior, theta=theta, init=init,
                          coarse_points=coarse_points, stop_rule=stop_rule, obj_atol=obj_atol, obj_rtol=obj_rtol,
                          calibrate=calibrate, linearization=linearization)
        D = pb.d * (pb.q + 1)
        dev = torch.device("cuda", self._device)
        mean = torch.empty((pb.N + 1, D), dtype=_dtype(pb.precision), device=dev)
        cov = torch.empty((pb.N + 1, D, D), dtype=_dtype(pb.precision), device=dev) if want_cov else None
        _check(self._L.parapn_server_submit(self._h, ctypes.byref(pb), int(req_id), _dptr(mean), _dptr(cov)))
        self._pending[int(req_id)] = (mean, cov)
        return mean

    def step(self):
        """One iteration for all active requests; returns (n_active, n_queued)."""
        na, nq = ctypes.c_int32(), ctypes.c_int32()
        _check(self._L.parapn_server_step(self._h, ctypes.byref(na), ctypes.byref(nq)))
        return na.value, nq.value

    def poll(self, max_records=1024):
        """List of completion dicts (req_id, status, iterations, final_delta,
        t_submit, t_start, t_done, start, mean, sqrtcov)."""
        buf = (Completion * max_records)()
        n = ctypes.c_int32()
        _check(self._L.parapn_server_poll(self._h, buf, max_records, ctypes.byref(n)))
        out = []
        for k in range(n.value):
            c = buf[k]
            mean, cov = self._pending.pop(c.req_id, (None, None))
            out.append({"req_id": c.req_id, "status": c.status, "iterations": c.iterations,
                        "final_delta": c.final_delta, "t_submit": c.t_submit, "t_start": c.t_start,
                        "t_done": c.t_done, "start": STARTS.get(c.start, c.start), "sigma_hat": c.sigma_hat,
                        "objective": c.objective, "mean": mean, "sqrtcov": cov})
        return out

    def clock(self):
        return self._L.parapn_server_clock()

    def stats(self):
        """{'used_bytes', 'peak_bytes', 'admitted', 'completed'}."""
        u, pk = ctypes.c_size_t(), ctypes.c_size_t()
        a, c = ctypes.c_int64(), ctypes.c_int64()
        _check(self._L.parapn_server_stats(self._h, ctypes.byref(u), ctypes.byref(pk), ctypes.byref(a),
                                           ctypes.byref(c)))
        return {"used_bytes": u.value, "peak_bytes": pk.value, "admitted": a.value, "completed": c.value}


    def close(self):
        if self._h is not None:
            self._L.parapn_server_destroy(self._h)
            self._h = None
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def server_footprint(field, params, y0, t0, t1, q, N, *, precision="fp32", d=None) -> int:
    """Bytes that server admission charges for this request."""
    pb = make_problem(field, params, y0, t0, t1, q, N, precision=precision, d=d)
    n = ctypes.c_size_t()
    _check(load_library().parapn_server_footprint(ctypes.byref(pb), ctypes.byref(n)))
    return n.value
