"""Dense engine (method-of-lines field, D = d(q+1) up to 192): parity of the
GPU solve with the oracle's sequential square-root filter and RTS smoother
(Alg. 2 with the same start, the same iterations and the same stopping
rule).

Tolerances (as for the row-per-lane engine's solves): FP64 E0 means and
covariances 1e-9 relative (to the largest entry), FP32 E0 means 1e-4
relative.  The derivative components of an iterated solve are compared
through the covariances and the E0 means they produce.  Covariances are
compared as Sigma = L L^T (the factor's column signs are not unique).  Shapes
cover one 16-wide tile and a ragged tail (D = 10, 15, 24, 48, 192), N = 1, 2, 3 and ragged N, and the
batch entry point (every instance bitwise equal to its solve alone).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2310_01145_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import torch

    import paper_2310_01145_amd as m

    assert torch.cuda.is_available()
    m.load_library()
    return m


def np_(t):
    return t.double().cpu().numpy()


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def sigma(L):
    L = np.asarray(L, dtype=np.float64)
    return L @ np.swapaxes(L, -1, -2)


def same(a, b):
    import torch

    iv = {4: torch.int32, 8: torch.int64}
    return a.shape == b.shape and torch.equal(a.view(iv[a.element_size()]), b.view(iv[b.element_size()]))


def spec_args(sp):
    return (sp["field"], sp["params"], sp["y0"], sp["t0"], sp["t1"], sp["q"], sp["N"])


FP64_CASES = [
    # d, q, N, fixed iterations
    (8, 2, 50, 3),    # D = 24: a full tile and a ragged one
    (3, 4, 37, 3),    # D = 15: one ragged tile
    (5, 1, 64, 2),    # D = 10
    (16, 2, 33, 2),   # D = 48
    (8, 3, 1, 2),     # one step
    (8, 2, 2, 2),
    (6, 2, 3, 2),
]


@pytest.mark.parametrize("d,q,N,k", FP64_CASES)
def test_dense_fp64_matches_oracle(pp, d, q, N, k):
    sp = workloads.mol(d=d, N=N, q=q, seed=d + N, t1=0.25)
    ref = oracle.ieks(*spec_args(sp), fixed_iters=k, want_cov=True)
    print("dense fp64 d=%d q=%d N=%d k=%d" % (d, q, N, k), flush=True)
    out = pp.solve(*spec_args(sp), precision="fp64", fixed_iters=k, want_cov=True)
    assert out["status"] == pp.OK and out["iterations"] == k
    S = q + 1
    assert rel(np_(out["mean"])[:, ::S], ref["mean"][:, ::S]) < 1e-9
    assert rel(sigma(np_(out["sqrtcov"])), sigma(ref["sqrtcov"])) < 1e-9
    np.testing.assert_allclose(out["deltas"], ref["deltas"], rtol=1e-6,
                               atol=1e-9 * np.abs(ref["mean"][:, ::S]).max())


def test_dense_fp64_converges_like_the_oracle(pp):
    sp = workloads.mol(d=8, N=200, q=2, seed=3)
    ref = oracle.ieks(*spec_args(sp), tol=1e-10, max_iter=20)
    out = pp.solve(*spec_args(sp), precision="fp64", tol=1e-10, max_iter=20)
    assert ref["status"] == 0 and out["status"] == pp.OK
    assert out["iterations"] == ref["iterations"]
    assert rel(np_(out["mean"])[:, ::3], ref["mean"][:, ::3]) < 1e-9


def test_dense_fp32_matches_oracle(pp):
    sp = workloads.mol(d=16, N=100, q=2, seed=5)
    ref = oracle.ieks(*spec_args(sp), tol=1e-10, max_iter=20)
    out = pp.solve(*spec_args(sp), precision="fp32", tol=1e-10, max_iter=20)
    assert out["status"] == pp.OK
    assert rel(np_(out["mean"])[:, ::3], ref["mean"][:, ::3]) < 1e-4


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_dense_d64_matches_oracle(pp, prec, tol):
    """The benchmark's state size: d = 64 grid points, q = 2, D = 192."""
    sp = workloads.mol(d=64, N=12, q=2, seed=7, t1=12.0 / 4096)
    ref = oracle.ieks(*spec_args(sp), fixed_iters=2, want_cov=True)
    print("dense d=64 %s" % prec, flush=True)
    out = pp.solve(*spec_args(sp), precision=prec, fixed_iters=2, want_cov=True)
    assert out["status"] == pp.OK
    assert rel(np_(out["mean"])[:, ::3], ref["mean"][:, ::3]) < tol
    if prec == "fp64":
        assert rel(sigma(np_(out["sqrtcov"])), sigma(ref["sqrtcov"])) < 1e-9
    else:
        S, R = sigma(np_(out["sqrtcov"]))[:, ::3, ::3], sigma(ref["sqrtcov"])[:, ::3, ::3]
        # the E0 block of the covariances (measured 4.8e-6)
        print("  E0 covariance rel err %.2e" % rel(S, R), flush=True)
        assert rel(S, R) < 1e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dense_batch_equals_alone(pp, prec):
    sp, y0s = workloads.mol_batch(B=3, d=8, N=40, q=2, t1=0.5)
    out = pp.solve_batch(sp["field"], sp["params"], y0s, sp["t0"], sp["t1"], sp["q"], sp["N"], precision=prec,
                         tol=1e-10, max_iter=20, want_cov=True)
    for b in range(3):
        a = pp.solve(sp["field"], sp["params"], y0s[b], sp["t0"], sp["t1"], sp["q"], sp["N"], precision=prec,
                     tol=1e-10, max_iter=20, want_cov=True)
        assert out["iterations"][b] == a["iterations"]
        assert same(out["mean"][b], a["mean"]), b
        assert same(out["sqrtcov"][b], a["sqrtcov"]), b


def test_batch_of_row_per_lane_field(pp):
    y0s = np.array([[0.01], [0.02], [0.05]])
    out = pp.solve_batch("logistic", [], y0s, 0.0, 10.0, 2, 300, precision="fp64", fixed_iters=4)
    for b in range(3):
        a = pp.solve("logistic", [], y0s[b], 0.0, 10.0, 2, 300, precision="fp64", fixed_iters=4)
        assert same(out["mean"][b], a["mean"])


def mol_residual(mean, nu, q):
    """max_n |E1 mu_n - f(E0 mu_n)| / max_n |f(E0 mu_n)| for the method-of-lines
    field: at the fixed point of the iteration the ODE holds at every grid
    point (the noiseless observation of Sec. 3.2.1)."""
    S = q + 1
    y, dy = mean[..., ::S], mean[..., 1::S]
    d = y.shape[-1]
    f = nu * d * d * (np.roll(y, 1, axis=-1) - 2 * y + np.roll(y, -1, axis=-1)) + y * (1 - y)
    return np.abs(dy - f).max() / np.abs(f).max()


def test_dense_full_size_batch(pp):
    """The benchmark's batch as bench.py runs it (16 instances, d = 64,
    D = 192, N = 4096, to tol 1e-10): beyond the oracle's reach, so checked by
    properties that hold at any size -- every instance converges, the ODE holds
    at every grid point of the converged mean, FP32 agrees with FP64 within
    1e-4 on E0."""
    sp, y0s = workloads.mol_batch(B=16)
    args = (sp["field"], sp["params"], y0s, sp["t0"], sp["t1"], sp["q"], sp["N"])
    print("dense full size fp32", flush=True)
    r32 = pp.solve_batch(*args, precision="fp32", tol=1e-10, max_iter=20)
    print("dense full size fp64", flush=True)
    r64 = pp.solve_batch(*args, precision="fp64", tol=1e-10, max_iter=20)
    assert r32["status"] == pp.OK and r64["status"] == pp.OK
    assert all(r32["converged"]) and all(r64["converged"])
    m32, m64 = np_(r32["mean"]), np_(r64["mean"])
    assert np.isfinite(m32).all() and np.isfinite(m64).all()
    assert mol_residual(m64, sp["params"][0], sp["q"]) < 1e-6
    assert mol_residual(m32, sp["params"][0], sp["q"]) < 1e-3
    assert rel(m32[..., ::3], m64[..., ::3]) < 1e-4


def test_dense_batch_isolates_a_non_finite_instance(pp):
    """An instance whose defect overflows FP32 (start at 1e20) turns
    non-finite in its first iteration and is frozen; the other instances of
    the batch run on and come out bitwise as alone."""
    sp, y0s = workloads.mol_batch(B=3, d=8, N=40, q=2, t1=0.5)
    y0s = y0s.copy()
    y0s[1, :] = 1e20
    out = pp.solve_batch(sp["field"], sp["params"], y0s, sp["t0"], sp["t1"], sp["q"], sp["N"], precision="fp32",
                         tol=1e-10, max_iter=20)
    assert out["status"] == pp.ENONFINITE
    assert out["iterations"][1] == 1
    for b in (0, 2):
        a = pp.solve(sp["field"], sp["params"], y0s[b], sp["t0"], sp["t1"], sp["q"], sp["N"], precision="fp32",
                     tol=1e-10, max_iter=20)
        assert a["status"] == pp.OK and out["iterations"][b] == a["iterations"]
        assert same(out["mean"][b], a["mean"]), b


_REF_CACHE = {}


def _ref(key, sp, k, want_cov):
    if key not in _REF_CACHE:
        _REF_CACHE[key] = oracle.ieks(*spec_args(sp), fixed_iters=k, want_cov=want_cov)
    return _REF_CACHE[key]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_dense_d64_at_128_steps_matches_oracle(pp, prec, tol):
    """d = 64 (D = 192) at the benchmark's step size and N = 128 steps: seven
    sweep levels each way, with a 2D x 2D = 384 x 384 triangularisation per
    general combine."""
    sp = workloads.mol(d=64, N=128, q=2, seed=7, t1=128.0 / 4096)
    ref = _ref("d64n128", sp, 2, True)
    print("dense d=64 N=128 %s" % prec, flush=True)
    out = pp.solve(*spec_args(sp), precision=prec, fixed_iters=2, want_cov=True)
    assert out["status"] == pp.OK
    e = rel(np_(out["mean"])[:, ::3], ref["mean"][:, ::3])
    S, R = sigma(np_(out["sqrtcov"])), sigma(ref["sqrtcov"])
    c = rel(S, R) if prec == "fp64" else rel(S[:, ::3, ::3], R[:, ::3, ::3])
    print("  E0 mean rel err %.2e, covariance rel err %.2e" % (e, c))
    assert e < tol
    # FP32: the E0 block of the covariances (measured 1.2e-5)
    assert c < (1e-9 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_dense_workgroup_stride_loop_matches_oracle(pp, prec, tol):
    """d = 8, q = 2 (D = 24), N = 4096 over [0, 1] (the benchmark's N and h):
    the first sweep level has 2048 pairs, more than the resident workgroups
    (1024 in FP32, 512 in FP64), so each workgroup strides over several
    pairs; twelve levels each way."""
    sp = workloads.mol(d=8, N=4096, q=2, seed=11, t1=1.0)
    ref = _ref("d8n4096", sp, 2, True)
    print("dense d=8 N=4096 %s" % prec, flush=True)
    out = pp.solve(*spec_args(sp), precision=prec, fixed_iters=2, want_cov=True)
    assert out["status"] == pp.OK
    e = rel(np_(out["mean"])[:, ::3], ref["mean"][:, ::3])
    print("  E0 mean rel err %.2e" % e)
    assert e < tol
    # FP32 delta_2: a difference of two iterates with ~1e-4-relative FP32
    # error each, gated relative to itself at 1e-2 (the means carry 1e-4)
    np.testing.assert_allclose(out["deltas"], ref["deltas"], rtol=(1e-6 if prec == "fp64" else 1e-2))
    if prec == "fp64":
        assert rel(sigma(np_(out["sqrtcov"])), sigma(ref["sqrtcov"])) < 1e-9
