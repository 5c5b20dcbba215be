"""Continuous-batching server (parapn_server_*): each request's result is the
same alone and in the mix, a non-finite neighbour does not leak into other
requests, and admission respects the slot and HBM-footprint limits.

A pack scans every request with its own chunking and its own tree of levels
(the launches of a level serve all requests that have it), so a request's
arithmetic does not depend on its neighbours: alone and in the mix, results
must be bitwise equal, in both precisions.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle

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


def same(a, b):
    """bitwise equality of two device tensors (NaN patterns included)"""
    import torch

    iv = {4: torch.int32, 8: torch.int64}
    return (a.shape == b.shape and a.dtype == b.dtype
            and torch.equal(a.view(iv[a.element_size()]), b.view(iv[b.element_size()])))


def relerr_e0(x, ref, q):
    x, ref = np.asarray(x)[:, :: q + 1], np.asarray(ref)[:, :: q + 1]
    return np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300)


def req(field, params, y0, t1, q, N, prec, k=0, tol=1e-10, max_iter=20):
    return dict(field=field, params=params, y0=y0, t0=0.0, t1=t1, q=q, N=N, precision=prec, fixed_iters=k,
                tol=tol, max_iter=max_iter)


def serve_all(pp, reqs, max_slots=64, budget=0, max_steps=2000):
    srv = pp.Server(max_slots=max_slots, budget=budget)
    for i, r in enumerate(reqs):
        srv.submit(i, **r)
    done = {}
    steps = 0
    while len(done) < len(reqs):
        srv.step()
        for c in srv.poll():
            done[c["req_id"]] = c
        steps += 1
        assert steps < max_steps, "server did not drain"
    stats = srv.stats()
    srv.close()
    return done, stats


def alone(pp, r):
    return pp.solve(r["field"], r["params"], r["y0"], r["t0"], r["t1"], r["q"], r["N"], precision=r["precision"],
                    fixed_iters=r["fixed_iters"], tol=r["tol"], max_iter=r["max_iter"])


MIX = [
    req("logistic", [], [0.01], 10.0, 2, 1000, "fp64", k=6),
    req("logistic", [], [0.01], 10.0, 3, 257, "fp64", k=6),
    req("van_der_pol", [1.0], [2.0, 0.0], 6.3, 2, 100, "fp64", k=6),
    req("rigid_body", [], [1.0, 0.0, 0.9], 20.0, 2, 150, "fp64", k=6),
    req("logistic", [], [0.02], 8.0, 2, 64, "fp64", k=6),
    req("logistic", [], [0.01], 10.0, 2, 513, "fp32", k=8),
    req("van_der_pol", [1.0], [2.0, 0.0], 6.3, 2, 300, "fp32", k=6),
    req("van_der_pol", [1.5], [1.0, 0.5], 5.0, 2, 77, "fp64", k=6),
    req("logistic", [], [0.01], 10.0, 2, 1, "fp64", k=3),
    req("logistic", [], [0.05], 10.0, 2, 9, "fp32", k=4),
]


def test_each_request_is_the_same_alone_and_in_the_mix(pp):
    done, stats = serve_all(pp, MIX)
    assert stats["admitted"] == len(MIX) and stats["completed"] == len(MIX) and stats["used_bytes"] == 0
    for i, r in enumerate(MIX):
        c = done[i]
        a = alone(pp, r)
        assert c["status"] == a["status"] == pp.OK, (i, c["status"], a["status"])
        assert c["iterations"] == a["iterations"] == r["fixed_iters"]
        assert c["final_delta"] == a["final_delta"]
        assert same(c["mean"], a["mean"]), (i, relerr_e0(np_(c["mean"]), np_(a["mean"]), r["q"]))


def test_served_fp64_matches_the_oracle(pp):
    r = req("logistic", [], [0.01], 10.0, 2, 1000, "fp64", tol=1e-10)
    ref = oracle.ieks("logistic", [], [0.01], 0.0, 10.0, 2, 1000, max_iter=20, tol=1e-10)
    done, _ = serve_all(pp, [r, MIX[2], MIX[5]])
    c = done[0]
    assert c["status"] == pp.OK and c["iterations"] == ref["iterations"]
    assert relerr_e0(np_(c["mean"]), ref["mean"], 2) < 1e-9


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_nonfinite_neighbour_does_not_leak(pp, prec):
    """A Lorenz request started at y0 = (1e20, 1e20, 1e20): its Taylor
    initial state is finite in FP64, but the vector field there (~1e40) is
    beyond the FP32 range, so in FP32 its first iteration turns non-finite.
    Rigid-body requests of the same (precision, d, q) share its pack and
    must come out bitwise as alone (in FP64 too, whatever the Lorenz request
    does there)."""
    q = 2
    good = [req("rigid_body", [], [1.0, 0.0, 0.9], 20.0, q, 150, prec, k=5),
            req("rigid_body", [], [0.5, 0.8, 0.2], 10.0, q, 333, prec, k=5)]
    bad = req("lorenz", [10.0, 28.0, 8.0 / 3.0], [1e20, 1e20, 1e20], 1.0, q, 500, prec, k=5)
    mix = [good[0], bad, good[1]]
    done, _ = serve_all(pp, mix)
    if prec == "fp32":
        assert done[1]["status"] == pp.ENONFINITE
        assert done[1]["iterations"] == 1
    for i in (0, 2):
        a = alone(pp, mix[i])
        assert done[i]["status"] == pp.OK
        assert np.isfinite(np_(done[i]["mean"])).all()
        assert same(done[i]["mean"], a["mean"])


def test_admission_by_hbm_footprint(pp):
    reqs = [req("logistic", [], [0.01 * (i + 1)], 10.0, 2, 4000, "fp32", k=4) for i in range(5)]
    fp = pp.server_footprint("logistic", [], [0.01], 0.0, 10.0, 2, 4000, precision="fp32")
    assert fp > 0
    budget = 2 * fp + fp // 2  # room for two requests at a time
    done, stats = serve_all(pp, reqs, budget=budget)
    assert stats["peak_bytes"] <= budget and stats["peak_bytes"] == 2 * fp
    ivals = sorted((c["t_start"], c["t_done"]) for c in done.values())
    for s, _ in ivals:
        live = sum(1 for s2, e2 in ivals if s2 <= s < e2)
        assert live <= 2
    # arrival order is kept
    starts = [done[i]["t_start"] for i in range(len(reqs))]
    assert starts == sorted(starts)


def test_admission_by_slots(pp):
    reqs = [req("logistic", [], [0.01], 10.0, 2, 200 + 50 * i, "fp64", k=3) for i in range(4)]
    done, _ = serve_all(pp, reqs, max_slots=1)
    order = sorted(done.values(), key=lambda c: c["t_start"])
    for a, b in zip(order, order[1:]):
        assert b["t_start"] >= a["t_done"]


def test_request_larger_than_budget_is_refused(pp):
    srv = pp.Server(max_slots=4, budget=1 << 16)
    with pytest.raises(pp.ParapnError) as e:
        srv.submit(0, "logistic", [], [0.01], 0.0, 10.0, 2, 100000, precision="fp32")
    assert e.value.code == pp.ENOMEM
    srv.close()


def test_late_arrival_joins_and_finishes_first(pp):
    """Continuous batching: a short request submitted while a long one is
    iterating is admitted at the next step, shares its iterations, and
    completes first; both results equal their solves alone."""
    long_r = req("logistic", [], [0.01], 10.0, 2, 20000, "fp32", k=12)
    short_r = req("logistic", [], [0.03], 10.0, 2, 300, "fp32", k=3)
    srv = pp.Server(max_slots=8)
    srv.submit(0, **long_r)
    done = {}
    for _ in range(2):
        srv.step()
        done.update({c["req_id"]: c for c in srv.poll()})
    srv.submit(1, **short_r)
    steps = 0
    while len(done) < 2:
        na, nq = srv.step()
        if steps == 0:
            assert na == 2 and nq == 0
        done.update({c["req_id"]: c for c in srv.poll()})
        steps += 1
        assert steps < 100
    srv.close()
    assert done[1]["t_done"] < done[0]["t_done"]
    assert done[1]["t_start"] < done[0]["t_done"]
    for i, r in ((0, long_r), (1, short_r)):
        assert same(done[i]["mean"], alone(pp, r)["mean"])


def test_damped_and_plain_requests_share_a_server(pp):
    """Damped requests (lm_sigma > 0) run in packs of their own; every
    request, damped or not, is bitwise the same as alone."""
    reqs = [req("logistic", [], [0.01], 10.0, 2, 300, "fp64", k=4),
            req("logistic", [], [0.02], 10.0, 2, 200, "fp64", k=4),
            req("van_der_pol", [1.0], [2.0, 0.0], 6.3, 3, 150, "fp32", k=3)]
    damped = [dict(r, lm_sigma=0.1) for r in reqs]
    mix = [reqs[0], damped[0], reqs[1], damped[1], damped[2], reqs[2]]
    srv = pp.Server(max_slots=16)
    for i, r in enumerate(mix):
        srv.submit(i, **r)
    done = {}
    while len(done) < len(mix):
        srv.step()
        done.update({c["req_id"]: c for c in srv.poll()})
    srv.close()
    for i, r in enumerate(mix):
        a = pp.solve(r["field"], r["params"], r["y0"], r["t0"], r["t1"], r["q"], r["N"], precision=r["precision"],
                     fixed_iters=r["fixed_iters"], lm_sigma=r.get("lm_sigma", 0.0))
        assert done[i]["status"] == pp.OK
        assert same(done[i]["mean"], a["mean"]), i
    # the damping acts
    assert not same(done[0]["mean"], done[1]["mean"])


def serve_on(pp, reqs, stream=None, max_slots=64):
    srv = pp.Server(max_slots=max_slots, stream=stream)
    for i, r in enumerate(reqs):
        srv.submit(i, **r)
    done = {}
    steps = 0
    while len(done) < len(reqs):
        srv.step()
        done.update({c["req_id"]: c for c in srv.poll()})
        steps += 1
        assert steps < 2000
    srv.close()
    return done


COARSE_MIX = [
    dict(req("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 100.0, 3, 6000, "fp64"), init="coarse"),
    dict(req("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 100.0, 3, 3001, "fp32"), init="coarse"),
    dict(req("lotka_volterra", [0.7, 1.2, 0.9, 1.1], [1.3, 0.8], 15.0, 2, 2500, "fp64"), init="coarse"),
    dict(req("lotka_volterra", [1.3, 0.6, 1.1, 0.8], [0.9, 1.7], 15.0, 4, 777, "fp64"), init="coarse",
         coarse_points=200),
    dict(req("lotka_volterra", [0.7, 1.2, 0.9, 1.1], [1.3, 0.8], 15.0, 3, 1500, "fp32"), init="coarse"),
    req("logistic", [], [0.01], 10.0, 2, 1000, "fp64"),
]


def test_coarse_start_requests_equal_their_solves(pp):
    """Requests that start from their coarse-grid start (computed at
    admission, one launch for all admitted requests of a (d, q)) converge and
    are bitwise the solve of each alone (parapn_solve with the same start)."""
    done = serve_on(pp, COARSE_MIX)
    for i, r in enumerate(COARSE_MIX):
        a = pp.solve(r["field"], r["params"], r["y0"], r["t0"], r["t1"], r["q"], r["N"], precision=r["precision"],
                     tol=r["tol"], max_iter=r["max_iter"], init=r.get("init", "constant"),
                     coarse_points=r.get("coarse_points", 0))
        c = done[i]
        assert c["start"] == a["start"] == ("coarse" if r.get("init") else "constant")
        assert c["status"] == a["status"] == pp.OK, (i, c["status"], a["status"])
        assert c["iterations"] == a["iterations"]
        assert same(c["mean"], a["mean"]), i


def test_graph_replays_equal_direct_launches(pp):
    """The same stream of requests served on the legacy default stream
    (every launch issued directly) and on the server's own stream (packs
    whose composition lasts replay a captured graph): bitwise the same, at
    every request -- every replay of every graph fed the next iteration."""
    import torch

    mix = MIX + COARSE_MIX
    a = serve_on(pp, mix, stream=torch.cuda.default_stream())
    b = serve_on(pp, mix)
    for i in range(len(mix)):
        assert a[i]["iterations"] == b[i]["iterations"]
        assert same(a[i]["mean"], b[i]["mean"]), i


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_served_covariances_equal_the_solve(pp, prec):
    """Requests that ask for covariances get the factors of their last
    linearisation, bitwise those of parapn_solve with want_cov; a neighbour
    without covariances shares the pack."""
    mix = [dict(req("logistic", [], [0.01], 10.0, 2, 700, prec, k=5), want_cov=True),
           req("logistic", [], [0.03], 10.0, 2, 300, prec, k=3),
           dict(req("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 50.0, 3, 2000, prec), init="coarse", want_cov=True)]
    done = serve_on(pp, mix)
    for i, r in enumerate(mix):
        a = pp.solve(r["field"], r["params"], r["y0"], r["t0"], r["t1"], r["q"], r["N"], precision=prec,
                     fixed_iters=r["fixed_iters"], tol=r["tol"], max_iter=r["max_iter"],
                     init=r.get("init", "constant"), want_cov=r.get("want_cov", False))
        c = done[i]
        assert same(c["mean"], a["mean"]), i
        if r.get("want_cov"):
            assert same(c["sqrtcov"], a["sqrtcov"]), i
        else:
            assert c["sqrtcov"] is None
