"""Served stream of IVP requests with Poisson arrivals.

Two ways of serving one seeded stream (field, q, N drawn per request, see
``workloads.served_stream``):

* plain: the FP64 solver, one request at a time in arrival order (FIFO).  Its
  service times are measured back to back; its latencies follow from the
  single-server FIFO recursion  finish_i = max(arrival_i, finish_{i-1}) +
  service_i, which is what a real-time replay would give.
* served: the continuous-batching server (parapn_server_*) in FP32 square-root
  form, replayed in real time: requests are submitted when their arrival time
  has passed, every server step runs one Gauss-Newton iteration for all
  admitted requests, completions are polled after each step.

Latency is completion minus arrival.  The served results are compared with
the plain FP64 results of the same request (E0 coordinates, relative to the
request's max |E0 mean|).

    python -m paper_2310_01145_amd.serve [--requests 4096] [--load 0.8]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import workloads


def arrival_times(n, qps, seed=1):
    """Poisson process: exponential gaps of mean 1/qps (seeded)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=n))


def _solve_args(r):
    return (r["field"], r["params"], r["y0"], r["t0"], r["t1"], r["q"], r["N"])


def run_plain(pp, torch, reqs, tol=1e-10, max_iter=20, precision="fp64", keep=None):
    """Service time, status and iterations of each request solved alone."""
    service, status, iters = [], [], []
    for i, r in enumerate(reqs):
        torch.cuda.synchronize()
        a = time.perf_counter()
        out = pp.solve(*_solve_args(r), precision=precision, tol=tol, max_iter=max_iter)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - a)
        status.append(out["status"])
        iters.append(out["iterations"])
        if keep is not None:
            keep(i, out["mean"])
    return np.array(service), np.array(status), np.array(iters)


def fifo_latency(arrivals, service):
    finish = np.empty_like(service)
    t = 0.0
    for i, (a, s) in enumerate(zip(arrivals, service)):
        t = max(t, a) + s
        finish[i] = t
    return finish - arrivals, finish[-1] - arrivals[0] if len(arrivals) else 0.0


def run_served(pp, torch, reqs, arrivals, precision="fp32", tol=1e-10, max_iter=20, max_slots=512,
               budget=64 << 30, on_done=None):
    """Real-time replay through the server.  Returns per-request latency,
    status, iterations, queueing delay, the makespan and server stats."""
    n = len(reqs)
    srv = pp.Server(max_slots=max_slots, budget=budget)
    lat = np.zeros(n)
    wait = np.zeros(n)
    status = np.zeros(n, dtype=np.int64)
    iters = np.zeros(n, dtype=np.int64)
    t0 = srv.clock()
    nxt, ndone, steps = 0, 0, 0
    active = queued = 0
    while ndone < n:
        now = srv.clock() - t0
        while nxt < n and arrivals[nxt] <= now:
            srv.submit(nxt, *_solve_args(reqs[nxt]), precision=precision, tol=tol, max_iter=max_iter)
            nxt += 1
            queued += 1
        if active == 0 and queued == 0:
            if nxt < n:
                time.sleep(max(0.0, arrivals[nxt] - (srv.clock() - t0)))
            continue
        active, queued = srv.step()
        steps += 1
        for c in srv.poll():
            i = c["req_id"]
            lat[i] = c["t_done"] - t0 - arrivals[i]
            wait[i] = c["t_start"] - t0 - arrivals[i]
            status[i] = c["status"]
            iters[i] = c["iterations"]
            if on_done is not None:
                on_done(i, c["mean"])
            ndone += 1
    makespan = srv.clock() - t0 - arrivals[0]
    stats = srv.stats()
    srv.close()
    return lat, status, iters, wait, makespan, steps, stats


def pct(x, p):
    return float(np.percentile(x, p)) if len(x) else None


def run(n_requests=4096, load=0.8, seed=0, max_slots=512, budget=64 << 30, tol=1e-10, max_iter=20,
        saturate=True):
    import torch

    import paper_2310_01145_amd as pp

    reqs = workloads.served_stream(n_requests, seed=seed)
    Ns = np.array([r["N"] for r in reqs])
    qs = np.array([r["q"] for r in reqs])
    ref_e0 = {}

    def keep_ref(i, mean):
        ref_e0[i] = mean[:, :: qs[i] + 1].clone()

    # warm-up: library load and first launches of each configuration
    for q in (2, 3, 4):
        pp.solve("logistic", [], [0.01], 0.0, 1.0, q, 64, precision="fp64", fixed_iters=1)
        pp.solve("logistic", [], [0.01], 0.0, 1.0, q, 64, precision="fp32", fixed_iters=1)
        pp.solve("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 1.0, q, 64, precision="fp64", fixed_iters=1)
        pp.solve("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 1.0, q, 64, precision="fp32", fixed_iters=1)
    service, st_p, it_p = run_plain(pp, torch, reqs, tol=tol, max_iter=max_iter, keep=keep_ref)
    print("serve: plain FP64 pass done (%.1f s of service)" % service.sum(), file=sys.stderr, flush=True)
    capacity = n_requests / service.sum()
    qps = load * capacity
    arr = arrival_times(n_requests, qps, seed=seed + 1)
    lat_p, span_p = fifo_latency(arr, service)

    errs = np.full(n_requests, np.nan)

    def compare(i, mean):
        a = mean[:, :: qs[i] + 1].double()
        b = ref_e0.pop(i)
        if torch.isfinite(a).all() and torch.isfinite(b).all():
            errs[i] = float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))

    lat_s, st_s, it_s, wait_s, span_s, steps, stats = run_served(pp, torch, reqs, arr, tol=tol, max_iter=max_iter,
                                                                 max_slots=max_slots, budget=budget,
                                                                 on_done=compare)
    print("serve: real-time served replay done (%.1f s)" % span_s, file=sys.stderr, flush=True)
    sat = None
    if saturate:
        # every request present at time 0: the server's own throughput
        z = np.zeros(n_requests)
        lat_z, st_z, it_z, _, span_z, steps_z, stats_z = run_served(pp, torch, reqs, z, tol=tol, max_iter=max_iter,
                                                                    max_slots=max_slots, budget=budget)
        sat = {"req_per_s": n_requests / span_z, "steps_x_iters_per_s": float((Ns * it_z).sum()) / span_z,
               "makespan_s": span_z, "server_steps": steps_z, "peak_admitted_bytes": stats_z["peak_bytes"],
               "p50_latency_s": pct(lat_z, 50), "p99_latency_s": pct(lat_z, 99)}
    both_ok = (st_s == pp.OK) & (st_p == pp.OK)
    work_p = float((Ns * it_p).sum())
    work_s = float((Ns * it_s).sum())

    def status_counts(st):
        names = {pp.OK: "ok", pp.MAXITER: "maxiter", pp.ENONFINITE: "nonfinite"}
        return {names.get(int(k), str(int(k))): int((st == k).sum()) for k in np.unique(st)}

    return {
        "workload": "served stream of %d IVP requests (logistic / FHN / LV, q in 2..4, N log-uniform 256..65536), "
                    "Poisson arrivals at %.2f x plain FP64 capacity" % (n_requests, load),
        "qps": qps,
        "plain_fp64_fifo": {
            "capacity_req_per_s": capacity,
            "req_per_s": n_requests / span_p,
            "steps_x_iters_per_s": work_p / span_p,
            "p50_latency_s": pct(lat_p, 50), "p99_latency_s": pct(lat_p, 99),
            "mean_service_s": float(service.mean()),
            "iterations_mean": float(it_p.mean()),
            "status": status_counts(st_p),
        },
        "served_fp32": {
            "req_per_s": n_requests / span_s,
            "steps_x_iters_per_s": work_s / span_s,
            "p50_latency_s": pct(lat_s, 50), "p99_latency_s": pct(lat_s, 99),
            "p50_queue_wait_s": pct(wait_s, 50), "p99_queue_wait_s": pct(wait_s, 99),
            "server_steps": steps,
            "iterations_mean": float(it_s.mean()),
            "peak_admitted_bytes": stats["peak_bytes"],
            "max_slots": max_slots, "budget_bytes": budget,
            "status": status_counts(st_s),
        },
        "served_fp32_saturated": sat,
        "fp32_vs_fp64_e0_relerr": {
            "compared": int(np.isfinite(errs[both_ok]).sum()),
            "max": float(np.nanmax(errs[both_ok])) if both_ok.any() else None,
            "p99": float(np.nanpercentile(errs[both_ok], 99)) if both_ok.any() else None,
            "within_1e-4": int((errs[both_ok] < 1e-4).sum()),
        },
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=4096)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-slots", type=int, default=512)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    a = ap.parse_args()
    out = run(a.requests, a.load, a.seed, a.max_slots, int(a.budget_gib * (1 << 30)))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
