"""Pins for the CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine used as an independent route (scipy's matrix exponential, numpy's QR),
exact rational arithmetic, dense joint-Gaussian conditioning, a closed-form
ODE solution, finite differences, or an algebraic identity (associativity,
Woodbury).  Each is chosen so that a plausible slip in the oracle (a dropped
term, a wrong sign or index, a transposed operand) makes one of them fail.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg
import scipy.special

import oracle

RNG = np.random.default_rng(20231001)


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ---------------------------------------------------------------------------
# Sec. 2.1: IWP(q) transition and process noise (closed form vs Van Loan)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("q", [1, 2, 3, 4])
@pytest.mark.parametrize("h", [0.5, 1.0, 1.7])
def test_iwp_matches_van_loan(q, h):
    """Phi(h), Q(h) of the IWP(q) SDE dY^(i) = Y^(i+1) dt, dY^(q) = dW, from the
    Van Loan matrix exponential expm([[F, L L^T], [0, -F^T]] h)."""
    S = q + 1
    F = np.diag(np.ones(q), 1)
    L = np.zeros((S, 1))
    L[-1, 0] = 1.0
    M = np.zeros((2 * S, 2 * S))
    M[:S, :S] = F
    M[:S, S:] = L @ L.T
    M[S:, S:] = -F.T
    E = scipy.linalg.expm(M * h)
    Phi_vl = E[:S, :S]
    Q_vl = E[:S, S:] @ Phi_vl.T
    Phi, Q = oracle.iwp(q, h)
    assert rel(Phi, Phi_vl) < 1e-12
    assert rel(Q, Q_vl) < 1e-11
    assert np.allclose(np.triu(Phi), Phi)  # reading of the garbled formula: upper triangular


@pytest.mark.parametrize("q", [1, 2, 3, 4])
@pytest.mark.parametrize("h", [1e-4, 0.01, 1.0])
def test_preconditioned_prior_is_step_independent(q, h):
    """Sec. 2.4 preconditioner: Phibar_ij = C(q-i, j-i), Qbar_ij = 1/(2q+1-i-j)
    in exact rationals, and sqrtQbar equals the exact LDL^T factor times sqrt(D)."""
    PhiB, sQB, T = oracle.precond_model(1, q, h)
    S = q + 1
    binom = np.array([[math.comb(q - i, j - i) if j >= i else 0 for j in range(S)] for i in range(S)], float)
    assert np.abs(PhiB - binom).max() < 1e-12 * binom.max()
    Qexact = [[Fraction(1, 2 * q + 1 - i - j) for j in range(S)] for i in range(S)]
    # exact LDL^T over the rationals
    Lr = [[Fraction(0)] * S for _ in range(S)]
    Dr = [Fraction(0)] * S
    for j in range(S):
        Dr[j] = Qexact[j][j] - sum(Lr[j][k] ** 2 * Dr[k] for k in range(j))
        Lr[j][j] = Fraction(1)
        for i in range(j + 1, S):
            Lr[i][j] = (Qexact[i][j] - sum(Lr[i][k] * Lr[j][k] * Dr[k] for k in range(j))) / Dr[j]
    chol_exact = np.array([[float(Lr[i][j]) * math.sqrt(float(Dr[j])) for j in range(S)] for i in range(S)])
    assert rel(sQB, chol_exact) < 1e-12
    Tref = np.array([math.sqrt(h) * h ** (q - i) / math.factorial(q - i) for i in range(S)])
    assert rel(T, Tref) < 1e-14


def test_kronecker_state_ordering():
    """State index k = i*(q+1) + j (the I_d (x) (q+1) ordering of Sec. 2.1)."""
    PhiB, sQB, T = oracle.precond_model(3, 2, 0.1)
    PB1, sQ1, T1 = oracle.precond_model(1, 2, 0.1)
    assert np.allclose(PhiB, np.kron(np.eye(3), PB1))
    assert np.allclose(sQB, np.kron(np.eye(3), sQ1))
    assert np.allclose(T, np.tile(T1, 3))


# ---------------------------------------------------------------------------
# vector fields: Jacobians by central differences
# ---------------------------------------------------------------------------
FIELD_CASES = [
    ("logistic", [], [0.3]),
    ("fhn", [0.2, 0.2, 3.0], [-1.1, 0.7]),
    ("lorenz", [10.0, 28.0, 8.0 / 3.0], [1.2, -0.4, 20.0]),
    ("lotka_volterra", [0.7, 1.2, 0.9, 1.1], [1.3, 0.8]),
    ("mol_heat_reaction", [0.01], list(0.5 + 0.1 * np.sin(2 * np.pi * np.arange(16) / 16))),
    ("rigid_body", [], [1.0, 0.2, 0.9]),
    ("van_der_pol", [1.0], [2.0, -0.3]),
]


@pytest.mark.parametrize("field,params,y", FIELD_CASES)
def test_jacobian_central_differences(field, params, y):
    y = np.array(y, float)
    J = oracle.field_jac(field, params, y)
    Jfd = np.zeros_like(J)
    for k in range(y.size):
        e = np.zeros_like(y)
        e[k] = 1e-6 * max(1.0, abs(y[k]))
        Jfd[:, k] = (oracle.field_f(field, params, y + e) - oracle.field_f(field, params, y - e)) / (2 * e[k])
    assert np.abs(J - Jfd).max() <= 1e-7 * max(1.0, np.abs(J).max())


def _ref_field(field, p):
    """Independent statements of the vector fields, written for objects with
    +, -, * (floats or numpy Polynomials); used by the Picard-iteration pin."""
    if field == "logistic":
        return lambda y: [y[0] * (1 - y[0])]
    if field == "fhn":
        a, b, c = p
        return lambda y: [c * (y[0] - y[0] * y[0] * y[0] * (1.0 / 3.0) + y[1]), (y[0] - a + b * y[1]) * (-1.0 / c)]
    if field == "lorenz":
        s, r, be = p
        return lambda y: [s * (y[1] - y[0]), y[0] * (r - y[2]) - y[1], y[0] * y[1] - be * y[2]]
    if field == "lotka_volterra":
        al, be, ga, de = p
        return lambda y: [al * y[0] - be * y[0] * y[1], de * y[0] * y[1] - ga * y[1]]
    if field == "rigid_body":
        return lambda y: [-2.0 * y[1] * y[2], 1.25 * y[0] * y[2], -0.5 * y[0] * y[1]]
    if field == "van_der_pol":
        (mu,) = p
        return lambda y: [y[1], mu * ((1 - y[0] * y[0]) * y[1] - y[0])]
    if field == "mol_heat_reaction":
        (nu,) = p

        def f(y):
            d = len(y)
            k = nu * d * d
            return [k * (y[i - 1] - 2.0 * y[i] + y[(i + 1) % d]) + y[i] * (1 - y[i]) for i in range(d)]

        return f
    raise KeyError(field)


@pytest.mark.parametrize("field,params,y", FIELD_CASES)
def test_field_values(field, params, y):
    f_ref = _ref_field(field, params)
    assert rel(oracle.field_f(field, params, y), np.array(f_ref(list(np.array(y, float))), float)) < 1e-14


# ---------------------------------------------------------------------------
# eq. mu0: exact initial derivatives
# ---------------------------------------------------------------------------
def test_mu0_logistic_closed_form():
    y = 0.01
    y1 = y * (1 - y)
    y2 = y1 * (1 - 2 * y)
    y3 = y2 * (1 - 2 * y) - 2 * y1 ** 2
    y4 = y3 * (1 - 2 * y) - 6 * y1 * y2
    mu0 = oracle.taylor_mu0("logistic", [], [y], 4)
    assert rel(mu0, [y, y1, y2, y3, y4]) < 1e-14


def test_mu0_affine_closed_form():
    d, q = 3, 4
    L = RNG.normal(size=(d, d))
    c = RNG.normal(size=d)
    y0 = RNG.normal(size=d)
    mu0 = oracle.taylor_mu0("affine", list(L.ravel()) + list(c), y0, q).reshape(d, q + 1)
    expect = [y0]
    v = L @ y0 + c
    for k in range(1, q + 1):
        expect.append(v)
        v = L @ v
    expect = np.array(expect).T
    assert rel(mu0, expect) < 1e-13


@pytest.mark.parametrize("field,params,y", FIELD_CASES)
def test_mu0_picard(field, params, y):
    """Taylor coefficients from Picard iteration y <- y0 + int_0^t f(y) in
    truncated polynomial arithmetic (independent of the oracle's recursion)."""
    from numpy.polynomial import Polynomial as Poly

    q = 4
    f = _ref_field(field, params)
    y0 = np.array(y, float)
    Y = [Poly([v]) for v in y0]
    for _ in range(q + 1):
        F = f(Y)
        Y = [Poly([y0[i]]) + Poly(np.asarray(F[i].coef if isinstance(F[i], Poly) else [F[i]])[: q + 1]).integ()
             for i in range(len(y0))]
        Y = [Poly(p.coef[: q + 1]) for p in Y]
    coef = np.zeros((len(y0), q + 1))
    for i, p in enumerate(Y):
        cc = p.coef[: q + 1]
        coef[i, : cc.size] = cc
    derivs = coef * np.array([math.factorial(k) for k in range(q + 1)])
    mu0 = oracle.taylor_mu0(field, params, y0, q).reshape(len(y0), q + 1)
    assert np.abs(mu0 - derivs).max() <= 1e-12 * max(1.0, np.abs(derivs).max())


# ---------------------------------------------------------------------------
# Sec. 3.1.2: tria
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,m", [(3, 6), (8, 16), (10, 10), (16, 16), (6, 3), (15, 30)])
def test_tria(n, m):
    M = RNG.normal(size=(n, m))
    L = oracle.tria(M)
    assert np.allclose(np.tril(L), L)
    assert np.all(np.diag(L) >= 0)
    assert rel(L @ L.T, M @ M.T) < 1e-13
    if m >= n:  # full row rank: unique, equals R^T of numpy's QR of M^T with signs fixed
        R = np.linalg.qr(M.T, mode="r")
        Lq = R.T * np.sign(np.diag(R))
        assert rel(L, Lq) < 1e-12


# ---------------------------------------------------------------------------
# ParaRTS target: sequential KF/RTS vs dense joint-Gaussian conditioning
# ---------------------------------------------------------------------------
def random_linear_model(D, dobs, N, rng, sigma0=True):
    Phi = np.eye(D) + 0.3 * rng.normal(size=(D, D))
    sQ = np.tril(rng.normal(size=(D, D))) * 0.5 + np.eye(D)
    mu0 = rng.normal(size=D)
    S0 = np.tril(rng.normal(size=(D, D))) * 0.3 if sigma0 else np.zeros((D, D))
    H = rng.normal(size=(N, dobs, D))
    dv = rng.normal(size=(N, dobs))
    return mu0, S0, Phi, sQ, H, dv


def dense_conditioning(mu0, S0, Phi, sQ, H, dv, upto=None, rstd=None):
    """Joint Gaussian of Y_0..N (Y0 = mu0 + S0 w0, Y_n = Phi Y_{n-1} + sQ w_n),
    conditioned on H_n Y_n = d_n for n = 1..upto (all when upto is None);
    rstd: optional per-row noise standard deviations of the observations."""
    N, dobs, D = H.shape
    upto = N if upto is None else upto
    nw = (N + 1) * D
    G = np.zeros(((N + 1) * D, nw))
    m = np.zeros((N + 1) * D)
    G[:D, :D] = S0
    m[:D] = mu0
    for n in range(1, N + 1):
        Pn = Phi[n - 1] if np.ndim(Phi) == 3 else Phi  # per-step transition (or constant)
        Qn = sQ[n - 1] if np.ndim(sQ) == 3 else sQ
        G[n * D:(n + 1) * D] = Pn @ G[(n - 1) * D:n * D]
        G[n * D:(n + 1) * D, n * D:(n + 1) * D] += Qn
        m[n * D:(n + 1) * D] = Pn @ m[(n - 1) * D:n * D]
    Sig = G @ G.T
    C = np.zeros((upto * dobs, (N + 1) * D))
    for n in range(1, upto + 1):
        C[(n - 1) * dobs:n * dobs, n * D:(n + 1) * D] = H[n - 1]
    dd = dv[:upto].ravel()
    S = C @ Sig @ C.T
    if rstd is not None:
        S = S + np.diag(np.tile(np.asarray(rstd, dtype=float) ** 2, upto))
    K = np.linalg.solve(S, C @ Sig).T
    mp = m + K @ (dd - C @ m)
    Sp = Sig - K @ C @ Sig
    return mp.reshape(N + 1, D), Sp


@pytest.mark.parametrize("D,dobs,N", [(3, 1, 5), (8, 2, 6)])
def test_time_varying_kf_rts_equals_dense_conditioning(D, dobs, N):
    """A model whose transition and process noise change every step (e.g. a
    non-uniform grid): the sequential smoother equals dense conditioning with
    the same per-step matrices, and differs from the constant model built from
    the first step's (so the per-step matrices are really used)."""
    rng = np.random.default_rng(7 * D + N)
    mu0, S0, Phi, sQ, H, dv = random_linear_model(D, dobs, N, rng)
    Phis = np.stack([Phi + 0.1 * rng.normal(size=(D, D)) for _ in range(N)])
    sQs = np.stack([np.tril(sQ + 0.1 * rng.normal(size=(D, D))) for _ in range(N)])
    mf, sPf, ms, sPs = oracle.kf_rts(mu0, S0, Phis, sQs, H, dv)
    m_all, S_all = dense_conditioning(mu0, S0, Phis, sQs, H, dv)
    for n in range(N + 1):
        assert rel(ms[n], m_all[n]) < 1e-10
        Pn = S_all[n * D:(n + 1) * D, n * D:(n + 1) * D]
        assert np.abs(sPs[n] @ sPs[n].T - Pn).max() < 1e-10 * max(1.0, np.abs(Pn).max())
    m_c = oracle.kf_rts(mu0, S0, Phis[0], sQs[0], H, dv)[2]
    assert rel(m_c, m_all) > 1e-3


@pytest.mark.parametrize("D,dobs,N", [(3, 1, 5), (4, 2, 6), (8, 2, 7)])
def test_kf_rts_equals_dense_conditioning(D, dobs, N):
    rng = np.random.default_rng(D * 100 + N)
    mu0, S0, Phi, sQ, H, dv = random_linear_model(D, dobs, N, rng)
    mf, sPf, ms, sPs = oracle.kf_rts(mu0, S0, Phi, sQ, H, dv)
    m_all, S_all = dense_conditioning(mu0, S0, Phi, sQ, H, dv)
    for n in range(N + 1):
        assert rel(ms[n], m_all[n]) < 1e-10
        Pn = S_all[n * D:(n + 1) * D, n * D:(n + 1) * D]
        assert np.abs(sPs[n] @ sPs[n].T - Pn).max() < 1e-10 * max(1.0, np.abs(Pn).max())
    for n in range(1, N + 1):
        m_n, S_n = dense_conditioning(mu0, S0, Phi, sQ, H, dv, upto=n)
        assert rel(mf[n], m_n[n]) < 1e-10
        Pn = S_n[n * D:(n + 1) * D, n * D:(n + 1) * D]
        assert np.abs(sPf[n] @ sPf[n].T - Pn).max() < 1e-10 * max(1.0, np.abs(Pn).max())
        # the Dirac observation holds exactly in the filtered marginal
        assert np.abs(H[n - 1] @ mf[n] - dv[n - 1]).max() < 1e-9 * max(1.0, np.abs(mf[n]).max())


def test_kf_rts_with_noisy_rows_equals_dense_conditioning():
    """Observation rows with noise (the damping rows of the Levenberg-Marquardt
    variant): sequential square-root filter/smoother vs dense conditioning."""
    D, dobs, N = 6, 4, 6
    rng = np.random.default_rng(17)
    mu0, S0, Phi, sQ, H, dv = random_linear_model(D, dobs, N, rng)
    rstd = np.array([0.0, 0.0, 0.7, 2.5])
    mf, sPf, ms, sPs = oracle.kf_rts(mu0, S0, Phi, sQ, H, dv, rstd=rstd)
    m_all, S_all = dense_conditioning(mu0, S0, Phi, sQ, H, dv, rstd=rstd)
    for n in range(N + 1):
        assert rel(ms[n], m_all[n]) < 1e-10
        Pn = S_all[n * D:(n + 1) * D, n * D:(n + 1) * D]
        assert np.abs(sPs[n] @ sPs[n].T - Pn).max() < 1e-10 * max(1.0, np.abs(Pn).max())
    m_3, _ = dense_conditioning(mu0, S0, Phi, sQ, H, dv, upto=3, rstd=rstd)
    assert rel(mf[3], m_3[3]) < 1e-10
    # zero noise is the noiseless filter
    a = oracle.kf_rts(mu0, S0, Phi, sQ, H, dv, rstd=np.zeros(dobs))
    b = oracle.kf_rts(mu0, S0, Phi, sQ, H, dv)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_damped_iterate_equals_regularised_linear_smoother():
    """One damped IEKS iteration = the linear smoother on the model linearised
    at the constant trajectory mu0 with the pseudo-observations E0 Y_n = E0 mu0
    of standard deviation lm_sigma / sqrt(h), built from the unpreconditioned
    closed forms and dense conditioning at tiny N."""
    field, params, y0, q, N, t1, lm = "fhn", [0.2, 0.2, 3.0], np.array([-1.0, 1.0]), 2, 5, 0.5, 0.3
    d, S = 2, q + 1
    D = d * S
    h = t1 / N
    Phi1, Q1 = oracle.iwp(q, h)
    Phi, Q = np.kron(np.eye(d), Phi1), np.kron(np.eye(d), Q1)
    mu0 = oracle.taylor_mu0(field, params, y0, q)
    E0 = np.zeros((d, D))
    E1 = np.zeros((d, D))
    for i in range(d):
        E0[i, i * S] = 1.0
        E1[i, i * S + 1] = 1.0
    y = E0 @ mu0
    J = oracle.field_jac(field, params, y)
    f = oracle.field_f(field, params, y)
    Hn = np.vstack([E1 - J @ E0, E0])
    dn = np.concatenate([f - J @ y, y])
    H = np.repeat(Hn[None], N, axis=0)
    dv = np.repeat(dn[None], N, axis=0)
    rstd = np.concatenate([np.zeros(d), np.full(d, lm / np.sqrt(h))])
    m_all, _ = dense_conditioning(mu0, np.zeros((D, D)), Phi, np.linalg.cholesky(Q), H, dv, rstd=rstd)
    r = oracle.ieks(field, params, y0, 0.0, t1, q, N, fixed_iters=1, want_cov=False, lm_sigma=lm)
    assert rel(r["mean"], m_all) < 1e-9
    plain = oracle.ieks(field, params, y0, 0.0, t1, q, N, fixed_iters=1, want_cov=False)
    assert rel(plain["mean"], m_all) > 1e-6  # the damping does act


def test_damping_keeps_the_fixed_point_and_vanishes_when_weak():
    a = oracle.ieks("logistic", [], [0.01], 0.0, 10.0, 2, 400, max_iter=40, tol=1e-12, want_cov=True)
    b = oracle.ieks("logistic", [], [0.01], 0.0, 10.0, 2, 400, max_iter=40, tol=1e-12, want_cov=True, lm_sigma=0.05)
    assert a["status"] == 0 and b["status"] == 0
    assert rel(b["mean"], a["mean"]) < 1e-9
    # the factors of a damped solve come from an undamped pass: the same posterior
    assert np.abs(b["sqrtcov"] @ b["sqrtcov"].transpose(0, 2, 1)
                  - a["sqrtcov"] @ a["sqrtcov"].transpose(0, 2, 1)).max() < 1e-9
    w = oracle.ieks("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 10.0, 3, 200, fixed_iters=3, want_cov=False,
                    lm_sigma=1e9)
    p = oracle.ieks("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 10.0, 3, 200, fixed_iters=3, want_cov=False)
    assert rel(w["mean"], p["mean"]) < 1e-8


# ---------------------------------------------------------------------------
# Sec. 3.1: paper-form elements and operators
# ---------------------------------------------------------------------------
def filter_elements(mu0, S0, Phi, sQ, H, dv):
    N, dobs, D = H.shape
    out = []
    for n in range(1, N + 1):
        if n == 1:
            out.append(oracle.filter_element(Phi, sQ, H[0], dv[0], mu0, S0, True))
        else:
            out.append(oracle.filter_element(Phi, sQ, H[n - 1], dv[n - 1], np.zeros(D), np.zeros((D, D)), False))
    return out


@pytest.mark.parametrize("D,dobs,N", [(3, 1, 6), (8, 2, 9)])
def test_filter_prefix_equals_sequential_filter(D, dobs, N):
    """Alg. 1 forward part: the cumulative (x)_f of the elements gives the
    filtering marginals m^f_n = b_{1:n}, sqrtP^f_n = sqrtC_{1:n}; A and J of
    every prefix vanish."""
    rng = np.random.default_rng(7 + D)
    mu0, S0, Phi, sQ, H, dv = random_linear_model(D, dobs, N, rng)
    mf, sPf, _, _ = oracle.kf_rts(mu0, S0, Phi, sQ, H, dv)
    els = filter_elements(mu0, S0, Phi, sQ, H, dv)
    acc = els[0]
    for n in range(1, N + 1):
        if n > 1:
            acc = oracle.filter_combine(acc, els[n - 1])
        A, b, sC, eta, sJ = acc
        assert rel(b, mf[n]) < 1e-10
        assert np.abs(sC @ sC.T - sPf[n] @ sPf[n].T).max() < 1e-10 * max(1, np.abs(sPf[n]).max() ** 2)
        assert np.abs(A).max() < 1e-12 and np.abs(eta).max() < 1e-12 and np.abs(sJ).max() < 1e-12


@pytest.mark.parametrize("D,dobs,N", [(3, 1, 6), (8, 2, 9)])
def test_smoother_suffix_equals_rts(D, dobs, N):
    """Alg. 1 backward part: the reverse cumulative (x)_s of the smoothing
    elements gives m^s_n = g_{n:N}, sqrtP^s_n = sqrtL_{n:N}."""
    rng = np.random.default_rng(11 + D)
    mu0, S0, Phi, sQ, H, dv = random_linear_model(D, dobs, N, rng)
    mf, sPf, ms, sPs = oracle.kf_rts(mu0, S0, Phi, sQ, H, dv)
    els = [oracle.smoother_element(Phi, sQ, mf[n], sPf[n], n == N) for n in range(1, N + 1)]
    acc = els[-1]
    for n in range(N, 0, -1):
        if n < N:
            acc = oracle.smoother_combine(els[n - 1], acc)
        E, g, sL = acc
        assert rel(g, ms[n]) < 1e-10
        assert np.abs(sL @ sL.T - sPs[n] @ sPs[n].T).max() < 1e-10 * max(1, np.abs(sPs[n]).max() ** 2)
        assert np.abs(E).max() < 1e-12


def random_fat_elements(D, dobs, k, rng):
    """Non-trivial filtering elements: aggregates of a few consecutive raw
    elements (so A, C, J are all full and no prefix structure is present)."""
    mu0, S0, Phi, sQ, H, dv = random_linear_model(D, dobs, 3 * k + 1, rng)
    els = filter_elements(mu0, S0, Phi, sQ, H, dv)[1:]
    out = []
    for i in range(k):
        a = els[3 * i]
        for j in (1, 2):
            a = oracle.filter_combine(a, els[3 * i + j])
        out.append(a)
    return out


def _cmp_filter(x, y, tol):
    A1, b1, sC1, e1, sJ1 = x
    A2, b2, sC2, e2, sJ2 = y
    assert rel(A1, A2) < tol
    assert rel(b1, b2) < tol
    assert rel(sC1 @ sC1.T, sC2 @ sC2.T) < tol
    assert rel(e1, e2) < tol
    assert rel(sJ1 @ sJ1.T, sJ2 @ sJ2.T) < tol


@pytest.mark.parametrize("D,dobs", [(3, 1), (6, 2), (8, 2)])
def test_filter_operator_associative(D, dobs):
    a, b, c = random_fat_elements(D, dobs, 3, np.random.default_rng(D))
    left = oracle.filter_combine(oracle.filter_combine(a, b), c)
    right = oracle.filter_combine(a, oracle.filter_combine(b, c))
    _cmp_filter(left, right, 1e-10)


@pytest.mark.parametrize("D,dobs", [(3, 1), (8, 2)])
def test_filter_operator_covariance_form(D, dobs):
    """The square-root operator equals the covariance-form operator obtained
    from it by the Woodbury identity:
      A = A_j (I + C_i J_j)^{-1} A_i,  b = A_j (I + C_i J_j)^{-1}(b_i + C_i eta_j) + b_j,
      C = A_j (I + C_i J_j)^{-1} C_i A_j^T + C_j,
      eta = A_i^T (I + J_j C_i)^{-1}(eta_j - J_j b_i) + eta_i,
      J = A_i^T (I + J_j C_i)^{-1} J_j A_i + J_i."""
    ai, aj = random_fat_elements(D, dobs, 2, np.random.default_rng(3 * D))
    Ai, bi, sCi, ei, sJi = ai
    Aj, bj, sCj, ej, sJj = aj
    Ci, Ji, Cj, Jj = sCi @ sCi.T, sJi @ sJi.T, sCj @ sCj.T, sJj @ sJj.T
    I = np.eye(D)
    M1 = np.linalg.inv(I + Ci @ Jj)
    M2 = np.linalg.inv(I + Jj @ Ci)
    ref = (Aj @ M1 @ Ai, Aj @ M1 @ (bi + Ci @ ej) + bj, Aj @ M1 @ Ci @ Aj.T + Cj,
           Ai.T @ M2 @ (ej - Jj @ bi) + ei, Ai.T @ M2 @ Jj @ Ai + Ji)
    A, b, sC, e, sJ = oracle.filter_combine(ai, aj)
    assert rel(A, ref[0]) < 1e-10
    assert rel(b, ref[1]) < 1e-10
    assert rel(sC @ sC.T, ref[2]) < 1e-10
    assert rel(e, ref[3]) < 1e-10
    assert rel(sJ @ sJ.T, ref[4]) < 1e-10


@pytest.mark.parametrize("D", [3, 8])
def test_smoother_operator_associative(D):
    rng = np.random.default_rng(100 + D)
    els = []
    for _ in range(3):
        E = rng.normal(size=(D, D)) * 0.5
        g = rng.normal(size=D)
        sL = np.tril(rng.normal(size=(D, D)))
        els.append((E, g, sL))
    a, b, c = els
    left = oracle.smoother_combine(oracle.smoother_combine(a, b), c)
    right = oracle.smoother_combine(a, oracle.smoother_combine(b, c))
    assert rel(left[0], right[0]) < 1e-12
    assert rel(left[1], right[1]) < 1e-12
    assert rel(left[2] @ left[2].T, right[2] @ right[2].T) < 1e-12
    # and the marginal composition it encodes: L_ij = E_i L_j E_i^T + L_i
    E, g, sL = oracle.smoother_combine(a, b)
    assert rel(sL @ sL.T, a[0] @ b[2] @ b[2].T @ a[0].T + a[2] @ a[2].T) < 1e-12


# ---------------------------------------------------------------------------
# Alg. 2: IEKS
# ---------------------------------------------------------------------------
def test_affine_ode_converges_in_one_iteration():
    """Sec. 3.1: for an affine vector field the linearisation is exact, so the
    first smoothing pass is already the fixed point."""
    d, q, N = 2, 2, 200
    L = np.array([[-0.5, 1.0], [-1.0, -0.3]])
    c = np.array([0.2, -0.1])
    r = oracle.ieks("affine", list(L.ravel()) + list(c), [1.0, 0.0], 0.0, 5.0, q, N, fixed_iters=3, want_cov=False)
    scale = np.abs(r["mean"]).max()
    assert r["deltas"][1] <= 1e-12 * scale
    assert r["deltas"][2] <= 1e-12 * scale
    # and the solution is accurate: compare with the exact affine flow
    t = np.linspace(0.0, 5.0, N + 1)
    ystar = -np.linalg.solve(L, c)
    exact = np.array([ystar + scipy.linalg.expm(L * tt) @ (np.array([1.0, 0.0]) - ystar) for tt in t])
    assert np.abs(r["mean"][:, [0, q + 1]] - exact).max() < 1e-6


@pytest.mark.parametrize("q", [1, 2, 3])
def test_logistic_convergence_order(q):
    """The MAP estimate converges polynomially to the true solution as h -> 0
    (Sec. 3.2.2); on the logistic closed form 1/(1 + (1/y0 - 1) e^{-t}) the
    observed rate is q + 1 at the grid points (above the order-q guarantee).
    The range stays above the FP64 floor."""
    Ns = {1: [1024, 2048, 4096], 2: [256, 512, 1024, 2048], 3: [256, 512, 1024]}[q]
    errs = []
    for N in Ns:
        r = oracle.ieks("logistic", [], [0.01], 0.0, 10.0, q, N, max_iter=40, tol=1e-13, want_cov=False)
        assert r["status"] == 0
        t = np.linspace(0.0, 10.0, N + 1)
        y = 1.0 / (1.0 + (1.0 / 0.01 - 1.0) * np.exp(-t))
        errs.append(np.abs(r["mean"][:, 0] - y).max())
    slopes = -np.diff(np.log2(errs))
    assert np.all(slopes > q + 0.5), slopes


def test_fixed_point_satisfies_ode_at_grid_points():
    """At convergence the Dirac constraints E1 mu_n = f(E0 mu_n) hold."""
    r = oracle.ieks("logistic", [], [0.01], 0.0, 10.0, 2, 1000, max_iter=20, tol=1e-10, want_cov=True)
    assert r["status"] == 0 and r["iterations"] <= 20
    m = r["mean"]
    resid = m[1:, 1] - m[1:, 0] * (1 - m[1:, 0])
    assert np.abs(resid).max() < 1e-8
    # the posterior covariance of E1 - F_y E0 is zero at the grid points (noiseless data)
    for n in (1, 500, 1000):
        y = m[n, 0]
        h = np.array([-(1 - 2 * y), 1.0, 0.0])
        P = r["sqrtcov"][n] @ r["sqrtcov"][n].T
        assert abs(h @ P @ h) <= 1e-10 * max(np.abs(P).max(), 1e-30) + 1e-30


def approx_jac(J, lin):
    """The Jacobian the linearisation uses (remark on approximate Jacobians,
    Sec. 3.2.1): EK1 keeps F_y, EK0 takes 0, DiagonalEK1 its diagonal."""
    if lin == "ek0":
        return np.zeros_like(J)
    if lin == "diag_ek1":
        return np.diag(np.diag(J))
    return J


@pytest.mark.parametrize("lin", ["ek1", "ek0", "diag_ek1"])
def test_ieks_iterate_equals_linear_smoother(lin):
    """Two IEKS iterations = the linear smoother on the model linearised at the
    constant trajectory mu0 (Alg. 2), then at that smoother's E0 means; built
    here independently from the unpreconditioned closed forms and dense
    conditioning at tiny N, with the Jacobian each linearisation uses."""
    field, params, y0, q, N, t1 = "fhn", [0.2, 0.2, 3.0], np.array([-1.0, 1.0]), 2, 5, 0.5
    d, S = 2, q + 1
    D = d * S
    h = t1 / N
    Phi1, Q1 = oracle.iwp(q, h)
    Phi, Q = np.kron(np.eye(d), Phi1), np.kron(np.eye(d), Q1)
    mu0 = oracle.taylor_mu0(field, params, y0, q)
    E0 = np.zeros((d, D))
    E1 = np.zeros((d, D))
    for i in range(d):
        E0[i, i * S] = 1.0
        E1[i, i * S + 1] = 1.0
    traj = np.repeat(mu0[None], N + 1, axis=0)
    for it in (1, 2):
        H = np.zeros((N, d, D))
        dv = np.zeros((N, d))
        for n in range(1, N + 1):
            y = E0 @ traj[n]
            J = approx_jac(oracle.field_jac(field, params, y), lin)
            H[n - 1] = E1 - J @ E0
            dv[n - 1] = oracle.field_f(field, params, y) - J @ y
        traj, _ = dense_conditioning(mu0, np.zeros((D, D)), Phi, np.linalg.cholesky(Q), H, dv)
        r = oracle.ieks(field, params, y0, 0.0, t1, q, N, fixed_iters=it, want_cov=False, linearization=lin)
        assert rel(r["mean"], traj) < 1e-9


def test_diagonal_ek1_is_ek1_for_a_decoupled_field():
    """With no diffusion the method-of-lines chain is d uncoupled logistic
    equations: F_y is diagonal, so DiagonalEK1 takes exactly EK1's steps,
    while EK0 (F_y ~ 0) does not."""
    y0 = [0.3, 0.5, 0.7, 0.45]
    kw = dict(fixed_iters=3, want_cov=False)
    r1 = oracle.ieks("mol_heat_reaction", [0.0], y0, 0.0, 1.0, 2, 40, linearization="ek1", **kw)
    r2 = oracle.ieks("mol_heat_reaction", [0.0], y0, 0.0, 1.0, 2, 40, linearization="diag_ek1", **kw)
    r0 = oracle.ieks("mol_heat_reaction", [0.0], y0, 0.0, 1.0, 2, 40, linearization="ek0", **kw)
    assert rel(r2["mean"], r1["mean"]) < 1e-14
    assert rel(r0["mean"], r1["mean"]) > 1e-6


@pytest.mark.parametrize("field,params,y0,t1,lin", [
    ("logistic", [], [0.01], 10.0, "ek0"),
    ("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 5.0, "diag_ek1"),
])
def test_approximate_jacobian_fixed_point_solves_the_ode(field, params, y0, t1, lin):
    """An approximate Jacobian changes the iteration, not what a fixed point
    satisfies: the noiseless constraints E1 mu_n = f(E0 mu_n) hold at every
    grid point, and the E0 means approximate the ODE solution as closely as
    EK1's fixed point does."""
    from scipy.integrate import solve_ivp
    q, N = 3, 200
    r = oracle.ieks(field, params, y0, 0.0, t1, q, N, max_iter=200, tol=1e-12, want_cov=False, linearization=lin)
    assert r["status"] == 0
    d, S = len(y0), q + 1
    m = r["mean"]
    for n in (1, N // 2, N):
        f = oracle.field_f(field, params, m[n, ::S])
        assert np.abs(m[n, 1::S] - f).max() < 1e-9
    t = np.linspace(0.0, t1, N + 1)
    fun = (lambda _t, y: oracle.field_f(field, params, np.asarray(y)))
    ref = solve_ivp(fun, (0.0, t1), y0, t_eval=t, rtol=1e-12, atol=1e-12, method="DOP853").y.T
    r1 = oracle.ieks(field, params, y0, 0.0, t1, q, N, max_iter=50, tol=1e-12, want_cov=False)
    e_lin, e_ek1 = np.abs(m[:, ::S] - ref).max(), np.abs(r1["mean"][:, ::S] - ref).max()
    assert e_lin < 3 * e_ek1 + 1e-10


@pytest.mark.parametrize("D,dobs", [(3, 1), (8, 2)])
def test_first_element_is_initial_state_combined_with_regular_element(D, dobs):
    """Reading used by the GPU scan: the paper's first element a_1 = p(Y1 | Z1)
    (built from m0 = mu0, P0 = Sigma0) equals the initial distribution, written
    as the element (A=0, b=mu0, sqrtC=sqrtSigma0, eta=0, sqrtJ=0), combined by
    (x)_f with the regular element of step 1 (built from m = 0, P = 0)."""
    rng = np.random.default_rng(5 * D)
    mu0, S0, Phi, sQ, H, dv = random_linear_model(D, dobs, 1, rng)
    first = oracle.filter_element(Phi, sQ, H[0], dv[0], mu0, S0, True)
    reg = oracle.filter_element(Phi, sQ, H[0], dv[0], np.zeros(D), np.zeros((D, D)), False)
    Z = np.zeros((D, D))
    state = (Z, mu0, S0, np.zeros(D), Z)
    comb = oracle.filter_combine(state, reg)
    assert np.abs(comb[0]).max() < 1e-12 and np.abs(comb[3]).max() < 1e-12 and np.abs(comb[4]).max() < 1e-12
    assert rel(comb[1], first[1]) < 1e-10
    assert rel(comb[2] @ comb[2].T, first[2] @ first[2].T) < 1e-10


@pytest.mark.parametrize("q", [1, 2, 3, 4])
@pytest.mark.parametrize("theta,h", [(0.5, 0.01), (2.0, 0.3), (1.0, 1e-3)])
def test_ioup_prior_matches_van_loan(q, theta, h):
    """IOUP(q, theta) blocks (the q-th derivative an Ornstein-Uhlenbeck
    process; the oracle integrates Q by quadrature) against Van Loan's block
    exponential evaluated in 40-digit arithmetic (in double precision its
    smallest Q entries cancel), entry by entry (Q scaled by sqrt(Q_ii Q_jj)),
    and the OU closed forms of the last block entries."""
    import mpmath

    Phi, Q = oracle.ioup(q, theta, h)
    S = q + 1
    with mpmath.workdps(40):
        C = mpmath.zeros(2 * S, 2 * S)
        for i in range(q):
            C[i, i + 1] = -h
            C[S + i + 1, S + i] = h
        C[q, q] = theta * h
        C[2 * S - 1, 2 * S - 1] = -theta * h
        C[q, S + q] = h
        E = mpmath.expm(C)
        E12 = E[:S, S:]
        Pm = E[S:, S:].T
        Qm = Pm * E12
        Pr = np.array([[float(Pm[i, j]) for j in range(S)] for i in range(S)])
        Qr = np.array([[float(Qm[i, j]) for j in range(S)] for i in range(S)])
    assert np.abs(Phi - Pr).max() < 1e-13 * np.abs(Pr).max()
    sc = np.sqrt(np.outer(np.diag(Qr), np.diag(Qr)))
    assert (np.abs(Q - Qr) / sc).max() < 1e-10
    assert abs(Phi[q, q] - np.exp(-theta * h)) < 1e-15
    assert abs(Q[q, q] - (1 - np.exp(-2 * theta * h)) / (2 * theta)) < 1e-14 * Q[q, q]


@pytest.mark.parametrize("q", [1, 2, 4])
def test_ioup_with_zero_rate_is_the_integrated_wiener_process(q):
    h = 0.05
    Phi, Q = oracle.ioup(q, 0.0, h)
    P0, Q0 = oracle.iwp(q, h)
    assert np.abs(Phi - P0).max() < 1e-14
    sc = np.sqrt(np.outer(np.diag(Q0), np.diag(Q0)))
    assert (np.abs(Q - Q0) / sc).max() < 1e-10


def matern_cov_blocks(q, lam, h):
    """P = Cov(X^(i), X^(j)) = (-1)^j k^(i+j)(0) and C(h) = Cov(X^(i)(t+h),
    X^(j)(t)) = (-1)^j k^(i+j)(h), and P - C P^-1 C^T, all in 40-digit
    arithmetic, for the autocovariance k of the stationary process with
    spectral density (lam^2 + w^2)^-(q+1) (unit-diffusion Matern,
    nu = q + 1/2), from its textbook closed form
    k(tau) = e^{-lam tau} / ((p-1)! (2 lam)^{2p-1})
             sum_{j<p} (p-1+j)! / (j! (p-1-j)!) (2 lam tau)^{p-1-j},  p = q+1."""
    import mpmath

    p, S = q + 1, q + 1
    with mpmath.workdps(40):
        lam = mpmath.mpf(lam)

        def k(t):
            s = sum(mpmath.factorial(p - 1 + j) / (mpmath.factorial(j) * mpmath.factorial(p - 1 - j))
                    * (2 * lam * t) ** (p - 1 - j) for j in range(p))
            return mpmath.exp(-lam * t) * s / (mpmath.factorial(p - 1) * (2 * lam) ** (2 * p - 1))

        d0 = [mpmath.diff(k, mpmath.mpf(0), n) for n in range(2 * S - 1)]
        dh = [mpmath.diff(k, mpmath.mpf(h), n) for n in range(2 * S - 1)]
        P = mpmath.matrix(S, S)
        C = mpmath.matrix(S, S)
        for i in range(S):
            for j in range(S):
                P[i, j] = (-1) ** j * d0[i + j]
                C[i, j] = (-1) ** j * dh[i + j]
        Qm = P - C * mpmath.inverse(P) * C.T
        f = lambda M: np.array([[float(M[i, j]) for j in range(S)] for i in range(S)])
        return f(P), f(C), f(Qm)


@pytest.mark.parametrize("q", [1, 2, 3, 4])
@pytest.mark.parametrize("ell,h", [(1.0, 0.1), (0.5, 0.4), (3.0, 0.05)])
def test_matern_prior_reproduces_the_matern_covariance(q, ell, h):
    """Matern(q + 1/2, ell) blocks against the Matern autocovariance k: a
    transition that reproduces the stationary process has Phi P = C(h) and
    Q = P - Phi P Phi^T = P - C P^-1 C^T (P, C as in matern_cov_blocks)."""
    Phi, Q = oracle.matern(q, ell, h)
    P, C, Qr = matern_cov_blocks(q, np.sqrt(2 * q + 1) / ell, h)
    sc = np.sqrt(np.outer(np.diag(P), np.diag(P)))
    assert (np.abs(Phi @ P - C) / sc).max() < 1e-11
    scq = np.sqrt(np.outer(np.diag(Qr), np.diag(Qr)))
    assert (np.abs(Q - Qr) / scq).max() < 1e-10


@pytest.mark.parametrize("q", [1, 3])
def test_matern_with_long_length_scale_approaches_the_integrated_wiener_process(q):
    """As ell grows the drift's coefficients lam^(q+1-k) binom(q+1, k) vanish
    and the Matern blocks tend to the IWP(q) blocks."""
    h = 0.05
    Phi, Q = oracle.matern(q, 1e7, h)
    P0, Q0 = oracle.iwp(q, h)
    assert np.abs(Phi - P0).max() < 1e-6
    sc = np.sqrt(np.outer(np.diag(Q0), np.diag(Q0)))
    assert (np.abs(Q - Q0) / sc).max() < 1e-6
    Phi2, _ = oracle.matern(q, 2.0, h)
    assert np.abs(Phi2 - P0).max() > 1e-4


# ---------------------------------------------------------------------------
# Stopping quantity (Sec. 3.2.2): delta_k from the returned iterates
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("field,params,y0,t1,q,N", [
    ("logistic", [], [0.01], 10.0, 2, 200),
    ("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 20.0, 3, 300),
    ("lorenz", [10.0, 28.0, 8.0 / 3.0], [1.0, 1.0, 1.0], 0.5, 4, 100),
])
def test_delta_is_the_e0_change_between_returned_iterates(field, params, y0, t1, q, N):
    """delta_k = max_n max_i |E0 (mu_n^(k) - mu_n^(k-1))| in original
    coordinates, recomputed here from the means the oracle returns after k-1
    and k iterations (the iterate before the first is the constant mu0, whose
    E0 part is y0).  A delta taken in preconditioned coordinates, over all
    derivatives, or against the wrong iterate fails this."""
    K = 4
    means = [np.tile(np.asarray(y0, float), (N + 1, 1))]
    hist = None
    for k in range(1, K + 1):
        r = oracle.ieks(field, params, y0, 0.0, t1, q, N, fixed_iters=k, want_cov=False)
        means.append(r["mean"][:, :: q + 1])
        hist = r["deltas"]
    assert len(hist) == K
    for k in range(1, K + 1):
        ref = np.abs(means[k] - means[k - 1]).max()
        assert abs(hist[k - 1] - ref) <= 1e-12 * max(ref, 1e-300) + 1e-15, (k, hist[k - 1], ref)
    # an earlier fixed count gives the same leading history (the iteration
    # does not depend on how many passes are requested)
    assert np.array_equal(oracle.ieks(field, params, y0, 0.0, t1, q, N, fixed_iters=2, want_cov=False)["deltas"],
                          hist[:2])


@pytest.mark.parametrize("logN", [12, 18])
def test_gauss_newton_from_the_constant_start_diverges_on_fitzhugh_nagumo(logN):
    """FitzHugh-Nagumo on [0, 100] from Alg. 2's constant start, sequential
    smoother: the first Gauss-Newton increment is O(1) (the solution of the
    linearisation at y0 over the whole span), and the second is already far
    larger -- the iteration is only locally convergent (remark on the
    convergence of the time-parallel IEKS), so the start, not the parallel
    scan, is what fails on this workload.  The increments are recomputed from
    the returned iterates, as in the test above."""
    N = 1 << logN
    args = ("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 100.0, 3, N)
    it1 = oracle.ieks(*args, fixed_iters=1, want_cov=False)
    it2 = oracle.ieks(*args, fixed_iters=2, want_cov=False)
    d1 = np.abs(it1["mean"][:, ::4] - np.array([-1.0, 1.0])).max()
    d2 = np.abs(it2["mean"][:, ::4] - it1["mean"][:, ::4]).max()
    assert 0.5 < d1 < 10.0
    assert abs(it2["deltas"][1] - d2) <= 1e-12 * d2
    assert d2 > 10.0 * d1
    if logN == 18:
        assert d2 > 1e9


# ---------------------------------------------------------------------------
# Starting trajectory from a coarse grid (remark on other initial
# trajectories, Sec. 3.2.2): coarse sequential EKS + prior bridge
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_iwp_bridge_is_the_hermite_interpolant(q):
    """Conditioned on the full states (q derivatives) at both ends, the IWP(q)
    mean between them minimises the integral of the squared (q+1)-th
    derivative, i.e. it is the Hermite interpolant of degree 2q+1 (scipy's
    BPoly.from_derivatives, an independent route)."""
    from scipy.interpolate import BPoly

    rng = np.random.default_rng(q)
    H = 0.37
    xa, xb = rng.normal(size=q + 1), rng.normal(size=q + 1)
    bp = BPoly.from_derivatives([0.0, H], [xa, xb])
    for tau in (0.0, 0.05, 0.2, 0.31, H):
        out = oracle.iwp_bridge(q, H, tau, xa, xb)
        ref = np.array([bp.derivative(j)(tau) if j else bp(tau) for j in range(q + 1)])
        # the bridge solves with Q(H), whose condition number grows steeply
        # with q (about 8e10 at q = 4 and H = 0.37)
        assert rel(out, ref) < 1e-8, (tau, out, ref)


def test_coarse_grid_rule():
    """s = ceil(N / M_target) fine steps per coarse step, M = ceil(N / s)."""
    assert oracle.coarse_grid(1000, 1024) == (1, 1000)
    assert oracle.coarse_grid(1 << 18, 1152) == (228, 1150)
    assert oracle.coarse_grid(4096, 1024) == (4, 1024)
    assert oracle.coarse_grid(4097, 1024) == (5, 820)
    for N in (1, 7, 1000, 4097, 65535):
        for Mt in (1, 3, 64, 1024):
            s, M = oracle.coarse_grid(N, Mt)
            assert M * s >= N > (M - 1) * s and M <= max(Mt, 1)
    assert oracle.default_coarse_points(1 << 18) == 1152 and oracle.default_coarse_points(300) == 300


def test_coarse_smoother_is_the_linear_smoother_for_an_affine_field():
    """For an affine field the EK1 linearisation is exact wherever it is taken,
    so the coarse extended smoother on the full grid (s = 1) is the plain
    Kalman/RTS smoother of the model, which one IEKS pass also computes."""
    L = np.array([[-0.5, 1.0], [-1.0, -0.3]])
    c = np.array([0.2, -0.1])
    p = list(L.ravel()) + list(c)
    st = oracle.coarse_start("affine", p, [1.0, 0.0], 0.0, 5.0, 2, 200, M_target=200)
    r = oracle.ieks("affine", p, [1.0, 0.0], 0.0, 5.0, 2, 200, fixed_iters=1, want_cov=False)
    assert rel(st, r["mean"]) < 1e-10


@pytest.mark.parametrize("field,params,y0,q", [("logistic", [], [0.3], 2), ("van_der_pol", [1.0], [2.0, 0.0], 3),
                                               ("lorenz", [10.0, 28.0, 8.0 / 3.0], [1.0, 1.0, 1.0], 2)])
def test_coarse_smoother_single_step_by_hand(field, params, y0, q):
    """One coarse step (M = 1), written out in covariance form with numpy: the
    prediction from (mu0, 0) is (Phi mu0, Q); the ODE is linearised at the
    predicted mean; the update conditions on Hbar x = Hbar m- + innovation;
    with Sigma0 = 0 the smoothed node 0 is mu0 and node 1 the filtered mean;
    fine points are the prior bridge between them."""
    from scipy.interpolate import BPoly

    t1, N = 0.05, 8
    d, S = len(y0), q + 1
    D = d * S
    Phi1, Q1 = oracle.iwp(q, t1)
    Phi, Q = np.kron(np.eye(d), Phi1), np.kron(np.eye(d), Q1)
    mu0 = oracle.taylor_mu0(field, params, y0, q)
    mp, Pp = Phi @ mu0, Q
    y = mp[::S]
    f = oracle.field_f(field, params, y)
    J = oracle.field_jac(field, params, y)
    E0 = np.zeros((d, D))
    E1 = np.zeros((d, D))
    for i in range(d):
        E0[i, i * S] = 1.0
        E1[i, i * S + 1] = 1.0
    Hm = E1 - J @ E0
    innov = f - E1 @ mp
    K = Pp @ Hm.T @ np.linalg.inv(Hm @ Pp @ Hm.T)
    m1 = mp + K @ innov
    st = oracle.coarse_start(field, params, y0, 0.0, t1, q, N, M_target=1)
    assert rel(st[0], mu0) < 1e-14
    assert rel(st[N], m1) < 1e-9
    ts = np.linspace(0.0, t1, N + 1)
    for i in range(d):
        bp = BPoly.from_derivatives([0.0, t1], [mu0[i * S:(i + 1) * S], m1[i * S:(i + 1) * S]])
        ref = bp(ts)
        assert np.abs(st[:, i * S] - ref).max() <= 1e-9 * max(np.abs(ref).max(), 1e-12)


@pytest.mark.parametrize("q", [2, 3])
def test_coarse_start_converges_to_the_logistic_solution(q):
    """Logistic ODE (closed form): the coarse-grid start approaches the exact
    solution as the coarse grid is refined, at a rate of order q or better
    (a filter at coarse step H is a method of order ~q)."""
    N, t1, y0 = 4096, 10.0, 0.01
    t = np.linspace(0.0, t1, N + 1)
    exact = 1.0 / (1.0 + (1.0 / y0 - 1.0) * np.exp(-t))
    errs = []
    for M in (64, 128, 256):
        st = oracle.coarse_start("logistic", [], [y0], 0.0, t1, q, N, M_target=M)
        errs.append(np.abs(st[:, 0] - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > q - 0.5), (errs, rates)
    assert errs[-1] < 1e-4


# ---------------------------------------------------------------------------
# Sec. 2.4 uncertainty calibration (quasi-MLE diffusion) and the objective
# value (eq. objective-value) of the stopping rule
# ---------------------------------------------------------------------------
def dense_quadratic_form(mu0, S0, Phi, sQ, H, dv):
    """(d - C m)^T (C Sigma C^T)^-1 (d - C m) for the stacked observations
    C Y = d of the joint Gaussian of Y_0..N -- the data's log-likelihood is
    -qf / (2 sigma^2) - (N dobs / 2) log sigma^2 + const when every covariance
    carries the diffusion sigma^2, so sigma-hat^2 = qf / (N dobs)."""
    N, dobs, D = H.shape
    G = np.zeros(((N + 1) * D, (N + 1) * D))
    m = np.zeros((N + 1) * D)
    G[:D, :D] = S0
    m[:D] = mu0
    for n in range(1, N + 1):
        Pn = Phi[n - 1] if np.ndim(Phi) == 3 else Phi  # per-step transition (or constant)
        Qn = sQ[n - 1] if np.ndim(sQ) == 3 else sQ
        G[n * D:(n + 1) * D] = Pn @ G[(n - 1) * D:n * D]
        G[n * D:(n + 1) * D, n * D:(n + 1) * D] += Qn
        m[n * D:(n + 1) * D] = Pn @ m[(n - 1) * D:n * D]
    C = np.zeros((N * dobs, (N + 1) * D))
    for n in range(1, N + 1):
        C[(n - 1) * dobs:n * dobs, n * D:(n + 1) * D] = H[n - 1]
    r = dv.ravel() - C @ m
    S = C @ G @ G.T @ C.T
    return float(r @ np.linalg.solve(S, r))


@pytest.mark.parametrize("D,dobs,N,sigma0", [(3, 1, 6, True), (8, 2, 7, False), (6, 3, 5, True)])
def test_innovation_quadratic_forms_equal_the_joint_quadratic_form(D, dobs, N, sigma0):
    """The sequential filter's innovations (prediction-error decomposition)
    against the dense joint Gaussian of all observations."""
    rng = np.random.default_rng(D * 31 + N)
    mu0, S0, Phi, sQ, H, dv = random_linear_model(D, dobs, N, rng, sigma0)
    qf = oracle.kf_rts(mu0, S0, Phi, sQ, H, dv, return_qf=True)[4]
    ref = dense_quadratic_form(mu0, S0, Phi, sQ, H, dv)
    assert abs(qf - ref) <= 1e-9 * abs(ref)


def test_sigma_hat_of_an_affine_solve_is_the_quasi_mle_of_its_linear_model():
    """For an affine field every linearisation is exact, so the IEKS's
    quasi-MLE is that of one linear model: sigma-hat^2 = qf / (N d) with qf
    the dense joint quadratic form of the preconditioned model (IWP(q) closed
    forms, observation rows E1 - (h/q) L E0 and offsets c / T1, built here)."""
    L = np.array([[-0.5, 1.0], [-1.0, -0.3]])
    c = np.array([0.2, -0.1])
    d, q, N, t1 = 2, 2, 7, 0.7
    h = t1 / N
    r = oracle.ieks("affine", list(L.ravel()) + list(c), [1.0, 0.0], 0.0, t1, q, N, fixed_iters=2, want_cov=False)
    S = q + 1
    T = np.array([math.sqrt(h) * h ** (q - i) / math.factorial(q - i) for i in range(S)])
    Phib = np.array([[math.comb(q - i, j - i) if j >= i else 0 for j in range(S)] for i in range(S)], float)
    Qb = np.array([[1.0 / (2 * q + 1 - i - j) for j in range(S)] for i in range(S)])
    Phi, sQ = np.kron(np.eye(d), Phib), np.kron(np.eye(d), np.linalg.cholesky(Qb))
    Tf = np.tile(T, d)
    mu0 = oracle.taylor_mu0("affine", list(L.ravel()) + list(c), [1.0, 0.0], q) / Tf
    H = np.zeros((N, d, d * S))
    dv = np.zeros((N, d))
    for n in range(N):
        for a in range(d):
            H[n, a, a * S + 1] = 1.0
            for b in range(d):
                H[n, a, b * S] -= (h / q) * L[a, b]
            dv[n, a] = c[a] / T[1]
    qf = dense_quadratic_form(mu0, np.zeros((d * S, d * S)), Phi, sQ, H, dv)
    assert abs(r["sigma2"] - qf / (N * d)) <= 1e-9 * qf / (N * d)


@pytest.mark.parametrize("q,prior,theta", [(1, "iwp", 0.0), (2, "iwp", 0.0), (3, "ioup", 0.7), (2, "matern", 1.5)])
def test_objective_is_the_negative_log_density_under_the_prior(q, prior, theta):
    """V = sum_n -log N(eta_n; Phi eta_{n-1}, Q) minus the normalising
    constants, with Phi, Q from the Van Loan exponential of the prior's SDE and
    scipy's Gaussian log-density; and V = 0 on a path that follows the prior
    mean."""
    from scipy.stats import multivariate_normal

    S, d, N, h = q + 1, 2, 6, 0.3
    F = np.diag(np.ones(q), 1)
    if prior == "matern":
        lam = np.sqrt(2 * q + 1) / theta
        F[q] = [-scipy.special.comb(q + 1, k) * lam ** (q + 1 - k) for k in range(S)]
    else:
        F[q, q] = -theta
    M = np.zeros((2 * S, 2 * S))
    M[:S, :S] = F
    M[q, S + q] = 1.0
    M[S:, S:] = -F.T
    E = scipy.linalg.expm(M * h)
    Phi1, Q1 = E[:S, :S], E[:S, S:] @ E[:S, :S].T
    rng = np.random.default_rng(q)
    tr = rng.normal(size=(N + 1, d * S))
    ref = 0.0
    for n in range(1, N + 1):
        for i in range(d):
            a, b = tr[n - 1, i * S:(i + 1) * S], tr[n, i * S:(i + 1) * S]
            mvn = multivariate_normal(mean=Phi1 @ a, cov=Q1)
            ref -= mvn.logpdf(b) + 0.5 * np.linalg.slogdet(2 * np.pi * Q1)[1]
    V = oracle.objective(tr, q, h, prior=prior, theta=theta)
    assert abs(V - ref) <= 1e-8 * abs(ref)
    path = np.zeros((N + 1, d * S))
    path[0] = rng.normal(size=d * S)
    for n in range(1, N + 1):
        for i in range(d):
            path[n, i * S:(i + 1) * S] = Phi1 @ path[n - 1, i * S:(i + 1) * S]
    assert abs(oracle.objective(path, q, h, prior=prior, theta=theta)) <= 1e-10 * np.abs(path).max() ** 2


def test_objective_history_and_the_objective_stopping_rule():
    """The oracle's objective after each iteration is V of the iterate it
    returns, and with the objective rule (Sec. 3.2.2; atol 1e-9, rtol 1e-6)
    the loop stops at the first iteration whose change meets it."""
    args = ("logistic", [], [0.01], 0.0, 10.0, 2, 400)
    full = oracle.ieks(*args, max_iter=30, tol=1e-12, want_cov=False, stop_rule=1)
    assert full["status"] == 0
    h = 10.0 / 400
    for k in (1, 3, 6):
        rk = oracle.ieks(*args, fixed_iters=k, want_cov=False)
        assert abs(full["objectives"][k - 1] - oracle.objective(rk["mean"], 2, h)) <= 1e-10 * abs(full["objectives"][k - 1])
    V = np.concatenate([[full["objective0"]], full["objectives"]])
    ok = np.abs(np.diff(V)) <= 1e-9 + 1e-6 * np.abs(V[1:])
    first = int(np.argmax(ok)) + 1
    r = oracle.ieks(*args, max_iter=30, tol=1e-12, want_cov=False, stop_rule=2)
    assert r["status"] == 0 and r["iterations"] == first < full["iterations"]
    both = oracle.ieks(*args, max_iter=30, tol=1e-12, want_cov=False, stop_rule=3)
    assert both["iterations"] == min(first, full["iterations"])
