"""Approximate Jacobians (EK0: F_y ~ 0, DiagonalEK1: F_y ~ diag F_y; remark on
linearizing with approximate Jacobians, Sec. 3.2.1) on the GPU against the
oracle run with the same linearisation, start, iterations and stopping rule.

* fixed-size fields (row-per-lane engine, the Jacobian masked per request);
* the method-of-lines chain, which under either approximation runs as d
  decoupled problems of state size q+1 (its factors are block diagonal).

Tolerances as for the EK1 solves: FP64 means and covariances 1e-9 relative
(to the largest entry), FP32 E0 means 1e-4 relative; sigma-hat and the
objective values (sums over the chain, accumulated by atomics in no fixed
order) 1e-9 relative in FP64.  The batch entry point returns for every
instance bitwise what the instance gets alone.
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


FIXED = [
    ("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 1.0, 3, 200, "ek0", "constant"),
    ("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 1.0, 3, 200, "diag_ek1", "constant"),
    ("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 5.0, 3, 200, "ek0", "coarse"),
    ("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 5.0, 3, 200, "diag_ek1", "coarse"),
    ("lorenz", [10.0, 28.0, 8.0 / 3.0], [1.0, 1.0, 1.0], 2.0, 4, 333, "diag_ek1", "coarse"),
    ("lotka_volterra", [1.0, 0.5, 1.2, 0.8], [1.0, 1.5], 4.0, 2, 97, "ek0", "coarse"),
]


@pytest.mark.parametrize("field,params,y0,t1,q,N,lin,init", FIXED)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fixed_size_fields_match_the_oracle(pp, field, params, y0, t1, q, N, lin, init, prec):
    """Three iterations from the constant start (Alg. 2) or the coarse-grid
    start: means, factors and deltas."""
    print("case", field, lin, init, prec, N, flush=True)
    ref = oracle.ieks(field, params, y0, 0.0, t1, q, N, fixed_iters=3, want_cov=True, linearization=lin, init=init)
    r = pp.solve(field, params, y0, 0.0, t1, q, N, precision=prec, fixed_iters=3, want_cov=True, linearization=lin,
                 init=init)
    assert r["iterations"] == 3
    S = q + 1
    if prec == "fp64":
        assert rel(np_(r["mean"]), ref["mean"]) < 1e-9
        assert rel(sigma(np_(r["sqrtcov"])), sigma(ref["sqrtcov"])) < 1e-9
        # delta is a difference of E0 values: its rounding is relative to them
        scale = np.abs(ref["mean"][:, ::S]).max()
        assert np.allclose(r["deltas"], ref["deltas"], rtol=1e-6, atol=1e-12 * scale), (r["deltas"], ref["deltas"])
    else:
        assert rel(np_(r["mean"])[:, ::S], ref["mean"][:, ::S]) < 1e-4


@pytest.mark.parametrize("field,params,y0,t1,q,N,lin,init", [
    ("logistic", [], [0.01], 10.0, 2, 1000, "ek0", "constant"),
    ("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 5.0, 3, 200, "diag_ek1", "coarse"),
    ("lotka_volterra", [1.0, 0.5, 1.2, 0.8], [1.0, 1.5], 4.0, 2, 97, "ek0", "coarse"),
])
def test_iterated_to_convergence_matches_the_oracle(pp, field, params, y0, t1, q, N, lin, init):
    """The full iteration (delta below 1e-10) takes the oracle's number of
    steps and reaches its fixed point."""
    kw = dict(max_iter=60, tol=1e-10, linearization=lin, init=init)
    ref = oracle.ieks(field, params, y0, 0.0, t1, q, N, want_cov=False, **kw)
    assert ref["status"] == 0
    r = pp.solve(field, params, y0, 0.0, t1, q, N, precision="fp64", **kw)
    assert r["status"] == pp.OK
    assert abs(r["iterations"] - ref["iterations"]) <= 1
    assert rel(np_(r["mean"]), ref["mean"]) < 1e-9


def test_diagonal_ek1_equals_ek1_for_diagonal_jacobians(pp):
    """Logistic (d = 1): the diagonal of F_y is F_y, so both give bitwise the
    same solve."""
    a = pp.solve("logistic", [], [0.01], 0.0, 10.0, 2, 500, precision="fp64", fixed_iters=4)
    b = pp.solve("logistic", [], [0.01], 0.0, 10.0, 2, 500, precision="fp64", fixed_iters=4, linearization="diag_ek1")
    assert same(a["mean"], b["mean"])


def mol_y0(d, seed=0):
    return workloads.mol_initial(d, seed)


MOL = [(8, 2, 40, "diag_ek1", 4), (16, 2, 256, "diag_ek1", 4), (16, 3, 101, "ek0", 2), (5, 1, 7, "diag_ek1", 3),
       (64, 2, 40, "diag_ek1", 3), (3, 4, 1, "diag_ek1", 2), (4, 2, 2, "ek0", 2), (6, 1, 4097, "diag_ek1", 2)]


@pytest.mark.parametrize("d,q,N,lin,its", MOL)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_decoupled_chain_matches_the_oracle(pp, d, q, N, lin, its, prec):
    """The method-of-lines chain under an approximate Jacobian (d decoupled
    problems on the GPU) against the oracle's full-state smoother: means,
    block-diagonal factors, deltas, sigma-hat and objective values."""
    y0 = mol_y0(d)
    print("case mol", d, q, N, lin, prec, flush=True)
    ref = oracle.ieks("mol_heat_reaction", [0.01], y0, 0.0, 1.0, q, N, fixed_iters=its, want_cov=True,
                      linearization=lin)
    r = pp.solve("mol_heat_reaction", [0.01], y0, 0.0, 1.0, q, N, precision=prec, fixed_iters=its, want_cov=True,
                 linearization=lin)
    assert r["iterations"] == its
    S = q + 1
    m = np_(r["mean"])
    if prec == "fp64":
        assert rel(m, ref["mean"]) < 1e-9
        C = np_(r["sqrtcov"])
        assert rel(sigma(C), sigma(ref["sqrtcov"])) < 1e-9
        # block diagonal: no factor entry couples two grid points
        mask = np.kron(np.eye(d), np.ones((S, S))) == 0
        assert np.abs(C[:, mask]).max() == 0.0
        assert np.allclose(r["deltas"], ref["deltas"], rtol=1e-6, atol=0)
        assert abs(r["sigma_hat"] ** 2 - ref["sigma2"]) <= 1e-9 * ref["sigma2"]
        assert np.allclose(r["objectives"], ref["objectives"], rtol=1e-9, atol=0)
    else:
        assert rel(m[:, ::S], ref["mean"][:, ::S]) < 1e-4


def test_decoupled_chain_objective_stop_rule(pp):
    """The objective-value rule (Sec. 3.2.2) stops the chain where the oracle
    stops."""
    d, q, N = 8, 2, 60
    y0 = mol_y0(d)
    kw = dict(max_iter=40, tol=1e-10, obj_atol=1e-9, obj_rtol=1e-6, linearization="diag_ek1")
    ref = oracle.ieks("mol_heat_reaction", [0.01], y0, 0.0, 1.0, q, N, want_cov=False,
                      stop_rule=oracle.STOP_OBJECTIVE, **kw)
    r = pp.solve("mol_heat_reaction", [0.01], y0, 0.0, 1.0, q, N, precision="fp64", stop_rule="objective", **kw)
    assert ref["status"] == 0 and r["status"] == pp.OK
    assert r["iterations"] == ref["iterations"]
    assert rel(np_(r["mean"]), ref["mean"]) < 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_decoupled_batch_equals_each_instance_alone(pp, prec):
    """Instances that stop at different iterations leave the pack with the
    result they get alone (means and factors, bitwise)."""
    d, q, N, B = 8, 2, 300, 4
    x = np.arange(d) / d
    y0s = np.stack([mol_y0(d), 0.9 + 0.01 * x, 0.5 + 0.4 * np.sin(2 * np.pi * x), 0.2 + 0.05 * np.cos(2 * np.pi * x)])
    kw = dict(precision=prec, max_iter=60, tol=1e-9, linearization="diag_ek1", want_cov=True)
    bt = pp.solve_batch("mol_heat_reaction", [0.01], y0s, 0.0, 1.0, q, N, **kw)
    if prec == "fp64":
        assert len(set(bt["iterations"])) > 1  # (the oracle takes 13, 12, 13, 13 iterations)
    for b in range(B):
        r = pp.solve("mol_heat_reaction", [0.01], y0s[b], 0.0, 1.0, q, N, **kw)
        assert bt["iterations"][b] == r["iterations"]
        assert same(bt["mean"][b], r["mean"])
        assert same(bt["sqrtcov"][b], r["sqrtcov"])


def test_decoupled_calibrated_fp32_sigma_hat(pp):
    """A calibrated FP32 chain takes sigma-hat from one FP64 filter pass at its
    final iterate: at convergence it matches the oracle's converged sigma-hat
    (1e-4, the FP32 iterate's own accuracy), and the factors scale by it; it is
    NaN without covariances."""
    d, q, N = 8, 2, 64
    y0 = mol_y0(d)
    kw = dict(max_iter=60, tol=1e-10, linearization="diag_ek1")
    ref = oracle.ieks("mol_heat_reaction", [0.01], y0, 0.0, 1.0, q, N, want_cov=False, **kw)
    a = pp.solve("mol_heat_reaction", [0.01], y0, 0.0, 1.0, q, N, precision="fp32", want_cov=True, calibrate=True,
                 **kw)
    u = pp.solve("mol_heat_reaction", [0.01], y0, 0.0, 1.0, q, N, precision="fp32", want_cov=True, **kw)
    assert ref["status"] == 0 and a["status"] == pp.OK
    sh = np.sqrt(ref["sigma2"])
    assert abs(a["sigma_hat"] - sh) <= 1e-4 * sh
    x, y = a["sqrtcov"].double(), u["sqrtcov"].double() * a["sigma_hat"]
    assert float((x - y).abs().max() / y.abs().max()) < 1e-6
    assert np.isnan(pp.solve("mol_heat_reaction", [0.01], y0, 0.0, 1.0, q, N, precision="fp32", **kw)["sigma_hat"])


def test_decoupled_chain_full_size(pp):
    """The method-of-lines batch at its full size (16 instances, d = 64,
    q = 2, N = 4096) under DiagonalEK1, iterated to delta < 1e-10: every
    instance converges, the FP64 fixed point satisfies the ODE at the grid
    points (the noiseless constraints; the remaining error of a linearly
    converging iteration is about delta / (1 - rate), times nu d^2 in E1), and
    the FP32 E0 means are within 1e-4 of the FP64 ones."""
    sp, y0s = workloads.mol_batch(B=16)
    d, q, N = 64, 2, 4096
    out = {}
    for prec in ("fp64", "fp32"):
        print("case mol full size", prec, flush=True)
        r = pp.solve_batch(sp["field"], sp["params"], y0s, 0.0, 1.0, q, N, precision=prec, max_iter=400, tol=1e-10,
                           linearization="diag_ek1")
        assert r["status"] == pp.OK and all(r["converged"])
        out[prec] = np_(r["mean"])
    m = out["fp64"]
    E0, E1 = m[:, 1:, 0::3], m[:, 1:, 1::3]
    k = sp["params"][0] * d * d
    f = k * (np.roll(E0, 1, -1) - 2 * E0 + np.roll(E0, -1, -1)) + E0 * (1 - E0)
    assert np.abs(E1 - f).max() < 1e-7 * max(np.abs(f).max(), 1.0)
    assert rel(out["fp32"][:, :, 0::3], m[:, :, 0::3]) < 1e-4


@pytest.mark.parametrize("where", ["host", "device"])
def test_decoupled_chain_from_a_given_trajectory(pp, where):
    """A caller's starting trajectory (original coordinates, host or device
    memory) is split over the chains: three DiagonalEK1 iterations from the
    EK1 fixed point equal the oracle's from the same start."""
    import torch

    d, q, N = 8, 2, 48
    y0 = mol_y0(d)
    start = oracle.ieks("mol_heat_reaction", [0.01], y0, 0.0, 1.0, q, N, max_iter=20, tol=1e-12,
                        want_cov=False)["mean"]
    start = start + 1e-3 * np.sin(np.arange(start.size)).reshape(start.shape)  # off the fixed point
    kw = dict(fixed_iters=3, linearization="diag_ek1")
    ref = oracle.ieks("mol_heat_reaction", [0.01], y0, 0.0, 1.0, q, N, want_cov=True, init_traj=start, **kw)
    init = torch.tensor(start, dtype=torch.float64, device="cuda") if where == "device" else start
    r = pp.solve("mol_heat_reaction", [0.01], y0, 0.0, 1.0, q, N, precision="fp64", want_cov=True, init_traj=init,
                 **kw)
    assert r["start"] == "given"
    assert rel(np_(r["mean"]), ref["mean"]) < 1e-9
    assert rel(sigma(np_(r["sqrtcov"])), sigma(ref["sqrtcov"])) < 1e-9
    assert np.allclose(r["deltas"], ref["deltas"], rtol=1e-6, atol=0)
