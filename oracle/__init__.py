"""Sequential FP64 CPU oracle for the parallel-in-time probabilistic ODE solver.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the HIP implementation: its arithmetic lives in
``oracle.c`` (plain C, built with gcc), and this module only marshals numpy
arrays through ctypes.

Functions follow the paper (Bosch et al., JMLR 2024):
  * ``iwp`` / ``precond_model``: IWP(q) transition and process noise in closed
    form (Sec. 2.1) and the coordinate-change preconditioner (Sec. 2.4).
  * ``taylor_mu0``: exact initial state mu0 (eq. mu0).
  * ``field_f`` / ``field_jac``: the vector-field registry.
  * ``tria``: the triangularisation operator (Sec. 3.1.2).
  * ``kf_rts``: sequential square-root Kalman filter + RTS smoother, the plain
    definition of what ParaRTS (Alg. 1) computes.
  * ``ieks``: Alg. 2 with that smoother.
  * ``filter_element`` / ``filter_combine`` / ``smoother_element`` /
    ``smoother_combine``: the paper's square-root elements and operators.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

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


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(ctypes.c_double)
        i, dl, l = ctypes.c_int, ctypes.c_double, ctypes.c_long
        L.orc_tria.argtypes = [i, i, P, P]
        L.orc_chol.argtypes = [i, P, P]
        L.orc_chol.restype = i
        L.orc_field_dim.argtypes = [i, i, i]
        L.orc_field_dim.restype = i
        L.orc_field_f.argtypes = [i, P, i, P, P]
        L.orc_field_jac.argtypes = [i, P, i, P, P]
        L.orc_taylor_mu0.argtypes = [i, P, i, P, i, P]
        L.orc_iwp.argtypes = [i, dl, P, P]
        L.orc_precond_diag.argtypes = [i, dl, P]
        L.orc_precond_model.argtypes = [i, i, dl, P, P, P]
        L.orc_kf_rts.argtypes = [i, i, l, P, P, P, P, P, P, P, P, P, P]
        L.orc_kf_rts.restype = i
        L.orc_ieks.argtypes = [i, P, i, i, P, dl, dl, i, l, i, dl, i, P, P, P, P, ctypes.POINTER(ctypes.c_int)]
        L.orc_ieks.restype = i
        L.orc_kf_rts_noise.argtypes = [i, i, l, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_kf_rts_noise.restype = i
        L.orc_ieks_lm.argtypes = [i, P, i, i, P, dl, dl, i, l, i, dl, i, P, dl, P, P, P,
                                  ctypes.POINTER(ctypes.c_int)]
        L.orc_ieks_lm.restype = i
        L.orc_ieks_prior.argtypes = [i, P, i, i, P, dl, dl, i, l, i, dl, i, P, dl, i, dl, P, P, P,
                                     ctypes.POINTER(ctypes.c_int)]
        L.orc_ieks_prior.restype = i
        L.orc_kf_rts_tv.argtypes = [i, i, l, P, P, P, P, P, P, P, P, P, P]
        L.orc_kf_rts_tv.restype = i
        L.orc_ioup.argtypes = [i, dl, dl, P, P]
        L.orc_ioup.restype = None
        L.orc_matern.argtypes = [i, dl, dl, P, P]
        L.orc_matern.restype = None
        L.orc_filter_element.argtypes = [i, i, P, P, P, P, P, P, i, P, P, P, P, P]
        L.orc_filter_combine.argtypes = [i] + [P] * 15
        L.orc_smoother_element.argtypes = [i, P, P, P, P, i, P, P, P]
        L.orc_smoother_combine.argtypes = [i] + [P] * 9
        LP = ctypes.POINTER(ctypes.c_long)
        L.orc_coarse_grid.argtypes = [l, l, LP, LP]
        L.orc_coarse_grid.restype = None
        L.orc_iwp_bridge.argtypes = [i, dl, dl, P, P, P]
        L.orc_iwp_bridge.restype = None
        L.orc_coarse_start.argtypes = [i, P, i, i, P, dl, dl, i, l, l, P]
        L.orc_coarse_start.restype = i
        L.orc_kf_rts_qf.argtypes = [i, i, l, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_kf_rts_qf.restype = i
        L.orc_objective.argtypes = [i, i, dl, l, P, i, dl]
        L.orc_objective.restype = dl
        L.orc_ieks_ext.argtypes = [i, P, i, i, P, dl, dl, i, l, i, dl, i, P, dl, i, dl, i, dl, dl, i, P, P, P, P,
                                   P, P, ctypes.POINTER(ctypes.c_int)]
        L.orc_ieks_ext.restype = i
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _field_id(field):
    return FIELDS[field] if isinstance(field, str) else int(field)


def tria(M):
    M = _f64(M)
    n, m = M.shape
    L = np.zeros((n, n))
    lib().orc_tria(n, m, _p(M), _p(L))
    return L


def chol(A):
    A = _f64(A)
    L = np.zeros_like(A)
    if lib().orc_chol(A.shape[0], _p(A), _p(L)) != 0:
        raise np.linalg.LinAlgError("matrix is not positive definite")
    return L


def field_dim(field, d, nparams):
    return lib().orc_field_dim(_field_id(field), d, nparams)


def field_f(field, params, y):
    y, p = _f64(y), _f64(params if len(params) else [0.0])
    f = np.zeros_like(y)
    lib().orc_field_f(_field_id(field), _p(p), y.size, _p(y), _p(f))
    return f


def field_jac(field, params, y):
    y, p = _f64(y), _f64(params if len(params) else [0.0])
    J = np.zeros((y.size, y.size))
    lib().orc_field_jac(_field_id(field), _p(p), y.size, _p(y), _p(J))
    return J


def taylor_mu0(field, params, y0, q):
    y0, p = _f64(y0), _f64(params if len(params) else [0.0])
    mu0 = np.zeros(y0.size * (q + 1))
    lib().orc_taylor_mu0(_field_id(field), _p(p), y0.size, _p(y0), q, _p(mu0))
    return mu0


def iwp(q, h):
    Phi = np.zeros((q + 1, q + 1))
    Q = np.zeros((q + 1, q + 1))
    lib().orc_iwp(q, float(h), _p(Phi), _p(Q))
    return Phi, Q


def precond_diag(q, h):
    T = np.zeros(q + 1)
    lib().orc_precond_diag(q, float(h), _p(T))
    return T


def precond_model(d, q, h):
    D = d * (q + 1)
    PhiB, sQB, T = np.zeros((D, D)), np.zeros((D, D)), np.zeros(D)
    lib().orc_precond_model(d, q, float(h), _p(PhiB), _p(sQB), _p(T))
    return PhiB, sQB, T


def kf_rts(mu0, S0, Phi, sqrtQ, H, dv, rstd=None, return_qf=False):
    """Sequential square-root KF + RTS.  H is [N, dobs, D], dv [N, dobs];
    Phi, sqrtQ are [D, D] (constant) or [N, D, D] (step n uses entry n-1);
    rstd (dobs) optional per-row observation noise standard deviations.
    Returns (mf, sPf, ms, sPs), stacks over n = 0..N; with return_qf (noiseless
    rows only) also the sum of the innovations' quadratic forms."""
    mu0, S0, Phi, sqrtQ, H, dv = map(_f64, (mu0, S0, Phi, sqrtQ, H, dv))
    N, dobs, D = H.shape
    mf, ms = np.zeros((N + 1, D)), np.zeros((N + 1, D))
    sPf, sPs = np.zeros((N + 1, D, D)), np.zeros((N + 1, D, D))
    if Phi.ndim == 3:
        assert Phi.shape == (N, D, D) and sqrtQ.shape == (N, D, D) and rstd is None and not return_qf
        rc = lib().orc_kf_rts_tv(D, dobs, N, _p(mu0), _p(S0), _p(Phi), _p(sqrtQ), _p(H), _p(dv), _p(mf), _p(sPf),
                                 _p(ms), _p(sPs))
        if rc != 0:
            raise FloatingPointError("non-finite values in the sequential smoother")
        return mf, sPf, ms, sPs
    if return_qf:
        assert rstd is None
        qf = ctypes.c_double(0.0)
        rc = lib().orc_kf_rts_qf(D, dobs, N, _p(mu0), _p(S0), _p(Phi), _p(sqrtQ), _p(H), _p(dv), _p(mf), _p(sPf),
                                 _p(ms), _p(sPs), ctypes.byref(qf))
        if rc != 0:
            raise FloatingPointError("non-finite values in the sequential smoother")
        return mf, sPf, ms, sPs, qf.value
    if rstd is None:
        rc = lib().orc_kf_rts(D, dobs, N, _p(mu0), _p(S0), _p(Phi), _p(sqrtQ), _p(H), _p(dv), _p(mf), _p(sPf),
                              _p(ms), _p(sPs))
    else:
        rs = _f64(rstd).ravel()
        assert rs.size == dobs
        rc = lib().orc_kf_rts_noise(D, dobs, N, _p(mu0), _p(S0), _p(Phi), _p(sqrtQ), _p(H), _p(dv), _p(rs),
                                    _p(mf), _p(sPf), _p(ms), _p(sPs))
    if rc != 0:
        raise FloatingPointError("non-finite values in the sequential smoother")
    return mf, sPf, ms, sPs


def ioup(q, theta, h):
    """IOUP(q, theta) blocks Phi(h), Q(h) in original coordinates."""
    S = q + 1
    Phi, Q = np.zeros((S, S)), np.zeros((S, S))
    lib().orc_ioup(q, float(theta), float(h), _p(Phi), _p(Q))
    return Phi, Q


def matern(q, ell, h):
    """Matern(q + 1/2, length scale ell) blocks Phi(h), Q(h) in original
    coordinates (unit diffusion)."""
    S = q + 1
    Phi, Q = np.zeros((S, S)), np.zeros((S, S))
    lib().orc_matern(q, float(ell), float(h), _p(Phi), _p(Q))
    return Phi, Q


PRIORS = {"iwp": 0, "ioup": 1, "matern": 2}


def coarse_grid(N, M_target):
    """(s, M): fine steps per coarse step and number of coarse steps."""
    s, M = ctypes.c_long(0), ctypes.c_long(0)
    lib().orc_coarse_grid(int(N), int(M_target), ctypes.byref(s), ctypes.byref(M))
    return s.value, M.value


def default_coarse_points(N):
    """Coarse-grid size used when none is given: max(1024, 64 ceil(log2 N)),
    at most N (the reading adopted for the O(log N) grid of the remark on
    other initial trajectories)."""
    lg = max(1, int(np.ceil(np.log2(max(N, 2)))))
    return int(min(N, max(1024, 64 * lg)))


def iwp_bridge(q, H, tau, xk, xk1):
    """IWP(q) prior mean at t_k + tau given the full states at t_k and t_k + H."""
    xk, xk1 = _f64(xk), _f64(xk1)
    out = np.zeros(q + 1)
    lib().orc_iwp_bridge(q, float(H), float(tau), _p(xk), _p(xk1), _p(out))
    return out


def coarse_start(field, params, y0, t0, t1, q, N, M_target=None, d=None):
    """Starting trajectory [N+1, D] (original coordinates) from a sequential
    extended Kalman smoother on a coarse grid, bridged to the fine grid by the
    prior.  Raises FloatingPointError if the coarse smoother diverged."""
    y0 = _f64(y0).ravel()
    params = _f64(params if len(params) else [0.0]).ravel()
    dd = y0.size if d is None else d
    fid = _field_id(field)
    dim = lib().orc_field_dim(fid, dd, params.size)
    if dim < 1:
        raise ValueError("field/parameter mismatch")
    M = default_coarse_points(N) if not M_target else int(M_target)
    out = np.zeros((N + 1, dim * (q + 1)))
    rc = lib().orc_coarse_start(fid, _p(params), params.size, dd, _p(y0), float(t0), float(t1), q, int(N), M,
                                _p(out))
    if rc == -1:
        raise ValueError("bad problem")
    if rc != 0:
        raise FloatingPointError("the coarse-grid smoother produced non-finite values")
    return out


def objective(traj, q, h, d=None, prior="iwp", theta=0.0):
    """V(eta) = 1/2 sum_n |eta_n - Phi eta_{n-1}|^2_{Q^-1} (eq. objective-value)
    of a trajectory [N+1, D] in original coordinates."""
    traj = _f64(traj)
    Np1, D = traj.shape
    dd = D // (q + 1) if d is None else d
    return lib().orc_objective(dd, q, float(h), Np1 - 1, _p(traj), PRIORS[prior], float(theta))


STOP_TRAJECTORY, STOP_OBJECTIVE = 1, 2
LINEARIZATIONS = {"ek1": 0, "ek0": 1, "diag_ek1": 2}


def ieks(field, params, y0, t0, t1, q, N, *, d=None, max_iter=20, tol=1e-10, fixed_iters=0, init_traj=None,
         want_cov=True, lm_sigma=0.0, prior="iwp", theta=0.0, init=None, coarse_points=0, stop_rule=1,
         obj_atol=1e-9, obj_rtol=1e-6, linearization="ek1"):
    """Alg. 2 with the sequential smoother.  Returns a dict with mean [N+1, D],
    sqrtcov [N+1, D, D] (original coordinates), status, iterations, deltas.
    lm_sigma > 0: Levenberg-Marquardt damping, a pseudo-observation of each
    step's E0 at the current iterate with std lm_sigma / sqrt(h).
    init="coarse": start from coarse_start(...) (coarse_points coarse steps,
    0 = the default) instead of the constant mu0.  stop_rule: bit 0 the
    trajectory change, bit 1 the objective change (|V_k - V_{k-1}| <=
    obj_atol + obj_rtol |V_k|), either stops.  The result also carries
    objectives (V after each iteration), objective0 (of the start) and sigma2
    (the quasi-MLE diffusion of the last undamped filter pass).
    linearization: "ek1" (exact Jacobian), "ek0" (F_y ~ 0) or "diag_ek1"
    (its diagonal) in every iteration (the coarse start uses EK1)."""
    if init == "coarse":
        init_traj = coarse_start(field, params, y0, t0, t1, q, N, coarse_points or None, d=d)
    y0 = _f64(y0).ravel()
    params = _f64(params if len(params) else [0.0]).ravel()
    dd = y0.size if d is None else d
    fid = _field_id(field)
    dim = lib().orc_field_dim(fid, dd, params.size)
    if dim < 1:
        raise ValueError("field/parameter mismatch")
    D = dim * (q + 1)
    mean = np.zeros((N + 1, D))
    cov = np.zeros((N + 1, D, D)) if want_cov else None
    hist = np.zeros(max(max_iter, fixed_iters, 1))
    iters = ctypes.c_int(0)
    init = _f64(init_traj) if init_traj is not None else None
    ohist = np.zeros_like(hist)
    obj0, s2 = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().orc_ieks_ext(fid, _p(params), params.size, dd, _p(y0), float(t0), float(t1), q, N, max_iter,
                            float(tol), fixed_iters, _p(init) if init is not None else None, float(lm_sigma),
                            PRIORS[prior], float(theta), int(stop_rule), float(obj_atol), float(obj_rtol),
                            LINEARIZATIONS[linearization], _p(mean),
                            _p(cov) if cov is not None else None, _p(hist), _p(ohist), ctypes.byref(obj0),
                            ctypes.byref(s2), ctypes.byref(iters))
    if rc == -1:
        raise ValueError("bad problem")
    k = iters.value
    return {"mean": mean, "sqrtcov": cov, "status": rc, "iterations": k, "deltas": hist[:k].copy(),
            "objectives": ohist[:k].copy(), "objective0": obj0.value, "sigma2": s2.value}


def filter_element(Phi, sqrtQ, H, dv, m_prev, sP_prev, first):
    Phi, sqrtQ, H, dv, m_prev, sP_prev = map(_f64, (Phi, sqrtQ, H, dv, m_prev, sP_prev))
    dobs, D = H.shape
    A, sC, sJ = np.zeros((D, D)), np.zeros((D, D)), np.zeros((D, D))
    b, eta = np.zeros(D), np.zeros(D)
    lib().orc_filter_element(D, dobs, _p(Phi), _p(sqrtQ), _p(H), _p(dv), _p(m_prev), _p(sP_prev), int(first),
                             _p(A), _p(b), _p(sC), _p(eta), _p(sJ))
    return A, b, sC, eta, sJ


def filter_combine(ai, aj):
    ai = [_f64(x) for x in ai]
    aj = [_f64(x) for x in aj]
    D = ai[1].size
    A, sC, sJ = np.zeros((D, D)), np.zeros((D, D)), np.zeros((D, D))
    b, eta = np.zeros(D), np.zeros(D)
    lib().orc_filter_combine(D, *[_p(x) for x in ai], *[_p(x) for x in aj], _p(A), _p(b), _p(sC), _p(eta), _p(sJ))
    return A, b, sC, eta, sJ


def smoother_element(Phi, sqrtQ, mf, sPf, last):
    Phi, sqrtQ, mf, sPf = map(_f64, (Phi, sqrtQ, mf, sPf))
    D = mf.size
    E, sL, g = np.zeros((D, D)), np.zeros((D, D)), np.zeros(D)
    lib().orc_smoother_element(D, _p(Phi), _p(sqrtQ), _p(mf), _p(sPf), int(last), _p(E), _p(g), _p(sL))
    return E, g, sL


def smoother_combine(bi, bj):
    bi = [_f64(x) for x in bi]
    bj = [_f64(x) for x in bj]
    D = bi[1].size
    E, sL, g = np.zeros((D, D)), np.zeros((D, D)), np.zeros(D)
    lib().orc_smoother_combine(D, *[_p(x) for x in bi], *[_p(x) for x in bj], _p(E), _p(g), _p(sL))
    return E, g, sL
