"""Served stream of IVP requests with Poisson arrivals.

Two ways of serving one seeded stream (field, q, N drawn per request, see
``workloads.served_stream``), every request from its coarse-grid start:

* plain: the FP64 solver (parapn_solve), one request at a time in arrival
  order, replayed in real time (a request that arrives while another is being
  solved waits).  A back-to-back pass first measures its capacity, which sets
  the arrival rate.
* served: the continuous-batching server (parapn_server_*) in FP32 square-root
  form, replayed in real time: requests are submitted when their arrival time
  has passed, every server step runs one Gauss-Newton iteration for all
  admitted requests, completions are polled after each step.

Latency is completion minus arrival.  The served results are compared with
the plain FP64 results of the same request (E0 coordinates, relative to the
request's max |E0 mean|).  Latencies and throughput are compared over the
requests that converge in both paths with the served result within 1e-4 of
the plain one; the status counts of each path are reported beside them.

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


def run_plain(pp, torch, reqs, tol=1e-10, max_iter=20, precision="fp64", keep=None, init="coarse"):
    """Service time, status and iterations of each request solved alone,
    back to back."""
    service, status, iters = [], [], []
    for i, r in enumerate(reqs):
        torch.cuda.synchronize()
        a = time.perf_counter()
        out = pp.solve(*_solve_args(r), precision=precision, tol=tol, max_iter=max_iter, init=init)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - a)
        status.append(out["status"])
        iters.append(out["iterations"])
        if keep is not None:
            keep(i, out["mean"])
    return np.array(service), np.array(status), np.array(iters)


def replay_plain(pp, torch, reqs, arrivals, tol=1e-10, max_iter=20, precision="fp64", init="coarse"):
    """Real-time replay of the plain solver, one request at a time in arrival
    order: returns per-request latency (completion minus arrival) and the
    makespan."""
    n = len(reqs)
    lat = np.zeros(n)
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        pp.solve(*_solve_args(r), precision=precision, tol=tol, max_iter=max_iter, init=init)
        torch.cuda.synchronize()
        lat[i] = time.perf_counter() - t0 - arrivals[i]
    return lat, time.perf_counter() - t0 - arrivals[0]


def run_served(pp, torch, reqs, arrivals, precision="fp32", tol=1e-10, max_iter=20, max_slots=512,
               budget=64 << 30, on_done=None, init="coarse"):
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
    step_s = []
    while ndone < n:
        now = srv.clock() - t0
        while nxt < n and arrivals[nxt] <= now:
            srv.submit(nxt, *_solve_args(reqs[nxt]), precision=precision, tol=tol, max_iter=max_iter, init=init)
            nxt += 1
            queued += 1
        if active == 0 and queued == 0:
            if nxt < n:
                time.sleep(max(0.0, arrivals[nxt] - (srv.clock() - t0)))
            continue
        a = time.perf_counter()
        active, queued = srv.step()
        step_s.append(time.perf_counter() - a)
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
    stats["step_ms_p50"] = 1e3 * pct(step_s, 50)
    stats["step_ms_p99"] = 1e3 * pct(step_s, 99)
    stats["step_ms_max"] = 1e3 * float(np.max(step_s)) if step_s else None
    return lat, status, iters, wait, makespan, steps, stats


def pct(x, p):
    return float(np.percentile(x, p)) if len(x) else None


def run(n_requests=4096, load=0.8, seed=0, max_slots=512, budget=64 << 30, tol=1e-10, max_iter=20,
        saturate=True, log=sys.stderr):
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
        for prec in ("fp64", "fp32"):
            pp.solve("logistic", [], [0.01], 0.0, 1.0, q, 64, precision=prec, fixed_iters=1, init="coarse")
            pp.solve("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 1.0, q, 64, precision=prec, fixed_iters=1,
                     init="coarse")
    service, st_p, it_p = run_plain(pp, torch, reqs, tol=tol, max_iter=max_iter, keep=keep_ref)
    print("serve: plain FP64 back-to-back pass done (%.1f s of service)" % service.sum(), file=log, flush=True)
    capacity = n_requests / service.sum()
    qps = load * capacity
    arr = arrival_times(n_requests, qps, seed=seed + 1)
    lat_p, span_p = replay_plain(pp, torch, reqs, arr, tol=tol, max_iter=max_iter)
    print("serve: plain FP64 real-time replay done (%.1f s)" % span_p, file=log, flush=True)

    errs = np.full(n_requests, np.nan)
    served_means = {}

    def keep_served(i, mean):
        # compared after the replay, so the comparison costs no replay time
        served_means[i] = mean

    lat_s, st_s, it_s, wait_s, span_s, steps, stats = run_served(pp, torch, reqs, arr, tol=tol, max_iter=max_iter,
                                                                 max_slots=max_slots, budget=budget,
                                                                 on_done=keep_served)
    print("serve: served FP32 real-time replay done (%.1f s)" % span_s, file=log, flush=True)
    for i, mean in served_means.items():
        a = mean[:, :: qs[i] + 1].double()
        b = ref_e0.pop(i)
        if torch.isfinite(a).all() and torch.isfinite(b).all():
            errs[i] = float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))
    served_means.clear()
    sat = None
    if saturate:
        # every request present at time 0: the server's own throughput
        z = np.zeros(n_requests)
        lat_z, st_z, it_z, _, span_z, steps_z, stats_z = run_served(pp, torch, reqs, z, tol=tol, max_iter=max_iter,
                                                                    max_slots=max_slots, budget=budget)
        print("serve: saturated served pass done (%.1f s)" % span_z, file=log, flush=True)
        sat = {"req_per_s": n_requests / span_z, "steps_x_iters_per_s": float((Ns * it_z).sum()) / span_z,
               "makespan_s": span_z, "server_steps": steps_z, "peak_admitted_bytes": stats_z["peak_bytes"],
               "p50_latency_s": pct(lat_z, 50), "p99_latency_s": pct(lat_z, 99)}
    both_ok = (st_s == pp.OK) & (st_p == pp.OK)
    same_acc = both_ok & (errs < 1e-4)
    work_p = float((Ns * it_p).sum())
    work_s = float((Ns * it_s).sum())

    def status_counts(st):
        names = {pp.OK: "ok", pp.MAXITER: "maxiter", pp.ENONFINITE: "nonfinite"}
        return {names.get(int(k), str(int(k))): int((st == k).sum()) for k in np.unique(st)}

    return {
        "workload": "served stream of %d IVP requests (logistic / FHN / LV, q in 2..4, N log-uniform 256..65536), "
                    "Poisson arrivals at %.2f x plain FP64 capacity, every request from its coarse-grid start"
                    % (n_requests, load),
        "qps": qps,
        "compared_requests": int(same_acc.sum()),
        "compared_on": "requests that converge in both paths with the served FP32 E0 means within 1e-4 of the "
                       "plain FP64 ones",
        "plain_fp64_fifo": {
            "capacity_req_per_s": capacity,
            "req_per_s": n_requests / span_p,
            "steps_x_iters_per_s": work_p / span_p,
            "p50_latency_s": pct(lat_p[same_acc], 50), "p99_latency_s": pct(lat_p[same_acc], 99),
            "p50_latency_s_all": pct(lat_p, 50), "p99_latency_s_all": pct(lat_p, 99),
            "mean_service_s": float(service.mean()),
            "iterations_mean": float(it_p.mean()),
            "status": status_counts(st_p),
        },
        "served_fp32": {
            "req_per_s": n_requests / span_s,
            "steps_x_iters_per_s": work_s / span_s,
            "p50_latency_s": pct(lat_s[same_acc], 50), "p99_latency_s": pct(lat_s[same_acc], 99),
            "p50_latency_s_all": pct(lat_s, 50), "p99_latency_s_all": pct(lat_s, 99),
            "p50_queue_wait_s": pct(wait_s, 50), "p99_queue_wait_s": pct(wait_s, 99),
            "server_steps": steps,
            "iterations_mean": float(it_s.mean()),
            "peak_admitted_bytes": stats["peak_bytes"],
            "step_ms_p50": stats["step_ms_p50"], "step_ms_p99": stats["step_ms_p99"], "step_ms_max": stats["step_ms_max"],
            "max_slots": max_slots, "budget_bytes": budget,
            "status": status_counts(st_s),
        },
        "served_fp32_saturated": sat,
        "fp32_vs_fp64_e0_relerr": {
            "both_converged": int(both_ok.sum()),
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
