"""Benchmark: ParaIEKS throughput on one MI355X.

One step = one complete solve (prior and initial state, then for every IEKS
iteration: linearisation, filtering elements, forward scan, smoothing
elements, reverse scan, convergence test; finally the output in original
coordinates) of the FitzHugh-Nagumo workload: d = 2, IWP(3) (D = 8),
N = 2^18 steps on t in [0, 100], started from the library's coarse-grid
trajectory (a sequential extended Kalman smoother on 1150 coarse steps,
bridged to the fine grid; computed inside the timed solve) and iterated to
Delta < 1e-10 (the FP32 path's threshold is max(1e-10, 2^-20 max|E0 mu|)), at
most 20 iterations.  From Alg. 2's constant start the Gauss-Newton iteration
diverges on this problem (in the sequential smoother too), which is reported
beside the figure.  value = N * iterations / seconds (time-steps x iterations
per second), whole job, FP32 square-root path.  Reported beside it: the FP64
path, a solve of 20 fixed iterations, the roofline of the dominant kernel of
the solve and of its iterations, the scan kernels at N = 2^18 and 2^20 (beyond
the Infinity Cache), an N sweep, the logistic latency, Lorenz-63 at D = 15,
the method-of-lines batch (EK1 on the dense engine; DiagonalEK1 as decoupled
chains), the served stream, and the oracle on the host (one thread, and one
instance per core).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-steps×iterations/sec per IEKS solve (FP32-sqrt vs FP64); p50/p99 latency"
UNIT = "time-steps*iterations/s"
PEAK = {"f32": 157.3e12, "f64": 78.6e12}  # MI355X vector FP32 / FP64 peak, FLOP/s
HBM_PEAK = 8.0e12


def workload(N, iters):
    """iters > 0: that many fixed iterations; 0: to Delta < 1e-10, at most 20."""
    return dict(field="fhn", params=[0.2, 0.2, 3.0], y0=[-1.0, 1.0], t0=0.0, t1=100.0, q=3, N=N, iters=iters)


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("scan_kernels.hip", "rowalg.h", "fields.h"):
        with open(os.path.join(ROOT, "paper_2310_01145_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, workload_tag):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), if it was taken
    on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "scan_kernels_%s_counters.md" % workload_tag)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"kernel_source_sha:\s*(\w+)", txt)
    m_b = re.search(r"traffic_bytes_per_launch %s:\s*([0-9.eE+]+)" % re.escape(kernel), txt)
    if not m_sha or not m_b or m_sha.group(1) != kernel_source_sha():
        return None
    return float(m_b.group(1))


def lorenz_workload(N, iters):
    return dict(field="lorenz", params=[10.0, 28.0, 8.0 / 3.0], y0=[1.0, 1.0, 1.0], t0=0.0, t1=20.0, q=4, N=N,
                iters=iters)


def logistic_latency(pp, torch, reps=100):
    """C0: the logistic problem (N = 1000, q = 2, constant start) solved to
    Delta < 1e-10 (at most 20 iterations), repeated; per-solve latency."""
    out = {}
    for prec in ("fp64", "fp32"):
        lat, it = [], []
        for i in range(reps + 3):
            torch.cuda.synchronize()
            a = time.perf_counter()
            r = pp.solve("logistic", [], [0.01], 0.0, 10.0, 2, 1000, precision=prec, tol=1e-10, max_iter=20)
            torch.cuda.synchronize()
            if i >= 3:
                lat.append(time.perf_counter() - a)
                it.append(r["iterations"])
        out[prec] = {"p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                     "iterations": int(np.median(it)), "status": r["status"], "solves": reps}
    return out


def n_sweep(pp, torch, iters, steps=3):
    """C1 throughput against N (FP32 and FP64), each solve from its own
    coarse-grid start."""
    out = []
    for e in range(12, 19):
        wl = workload(1 << e, iters)
        row = {"N": 1 << e}
        for prec in ("fp32", "fp64"):
            r = run_gpu(pp, torch, wl, prec, steps, 1, False)
            row[prec] = {"value": r["value"], "ms_per_solve": r["ms_per_step"], "status": r["status"][0],
                         "iterations": r["iterations_per_solve"][0]}
        out.append(row)
    return out


def beyond_cache(pp, torch, e=20):
    """The step-level scan kernels at N = 2^e (FP32, 3 fixed iterations from
    the coarse start): there the smoothing elements that k_fwd_down1 writes
    and the reverse-scan kernels read (about 100 B per step) no longer fit the
    256 MB Infinity Cache, so the algorithmic GB/s are HBM figures."""
    wl = workload(1 << e, 3)
    r = run_gpu(pp, torch, wl, "fp32", 2, 1, True)
    out = {"N": wl["N"], "iterations": 3, "status": r["status"][0], "ms_per_solve": r["ms_per_step"],
           "kernels": scan_kernel_table(r["profile_untimed"], wl, "fp32")}
    return out


def constant_start(pp, wl, prec):
    """Outcome of the same solve from the constant initial trajectory."""
    r = pp.solve(wl["field"], wl["params"], wl["y0"], wl["t0"], wl["t1"], wl["q"], wl["N"], precision=prec,
                 fixed_iters=wl["iters"], tol=1e-10, max_iter=20, init="constant")
    return {"status": r["status"], "iterations": r["iterations"], "final_delta": r["final_delta"],
            "deltas_first": [float(x) for x in r["deltas"][:4]]}


def run_gpu(pp, torch, wl, prec, steps, warmup, profile, d=2, init_traj=None):
    """Warm-up, then (profile) one untimed solve with every kernel timed by
    events, then the timed solves, during which only the dominant kernel of
    that pass carries events (so the timer does not slow the other launches).
    Without init_traj every solve computes its coarse-grid start itself."""
    D = d * (wl["q"] + 1)
    dt = torch.float32 if prec == "fp32" else torch.float64
    mean = torch.empty((wl["N"] + 1, D), dtype=dt, device="cuda")
    kw = dict(precision=prec, out=(mean, None), init_traj=init_traj, init="coarse")
    if wl["iters"] > 0:
        kw["fixed_iters"] = wl["iters"]
    else:
        kw.update(tol=1e-10, max_iter=20)
    args = (wl["field"], wl["params"], wl["y0"], wl["t0"], wl["t1"], wl["q"], wl["N"])
    for _ in range(warmup):
        pp.solve(*args, **kw)
    torch.cuda.synchronize()
    prof_all = dominant = None
    if profile:
        pp.profile_enable(True)
        pp.solve(*args, **kw)
        torch.cuda.synchronize()
        prof_all = pp.profile_read()
        dominant = max(prof_all, key=lambda k: prof_all[k][0])
        pp.profile_enable(True)
        pp.profile_only(dominant)
    lat, iters, statuses = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        r = pp.solve(*args, **kw)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
        iters.append(r["iterations"])
        statuses.append(r["status"])
        starts = r["start"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = None
    if profile:
        prof = pp.profile_read()
        pp.profile_only(None)
        pp.profile_enable(False)
    return {
        "value": wl["N"] * float(sum(iters)) / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "latency_ms_p50": 1e3 * float(np.percentile(lat, 50)),
        "latency_ms_p99": 1e3 * float(np.percentile(lat, 99)),
        "iterations_per_solve": iters,
        "status": statuses,
        "final_delta": r["final_delta"],
        "start": starts,
        "profile": prof,
        "profile_untimed": prof_all,
    }


def roofline(prof, wl, prec, prof_all=None):
    from paper_2310_01145_amd import costmodel

    d, q, N = 2, wl["q"], wl["N"]
    esize = 4 if prec == "fp32" else 8
    b1 = costmodel.forward_chunk(N)
    per = costmodel.per_step(d, q, esize, b1)
    # dominant kernel by total time
    name = max(prof, key=lambda k: prof[k][0])
    total_ms, launches = prof[name]
    avg_s = total_ms * 1e-3 / launches
    steps_per_launch = N if name in per else None
    ref = prof_all if prof_all else prof
    out = {"kernel": name, "avg_launch_us": avg_s * 1e6, "launches": launches,
           "share_of_kernel_time": ref[name][0] / sum(v[0] for v in ref.values())}
    if name == "coarse_eks":
        # one wavefront runs the sequential coarse filter and smoother in FP64:
        # a recursion bound by instruction latency, priced against the FP64 peak
        M = costmodel.coarse_points(N)
        fl = costmodel.coarse_step_flops(d, q) * M
        out.update({"bound": "alu", "achieved": fl / avg_s / 1e12, "peak": PEAK["f64"] / 1e12, "unit": "TFLOP/s",
                    "frac": fl / avg_s / PEAK["f64"], "traffic": stored_traffic(name, "fhn_n%d_%s" % (N, prec)),
                    "coarse_steps": M, "us_per_coarse_step": avg_s * 1e6 / M,
                    "note": "sequential recursion on one wavefront (one SIMD of 1024); its FP64 work per step is "
                            "%d flop" % costmodel.coarse_step_flops(d, q)})
        return out
    if steps_per_launch is None:
        out.update({"bound": "alu", "achieved": None, "peak": PEAK["f32" if esize == 4 else "f64"] / 1e12,
                    "unit": "TFLOP/s", "frac": None, "traffic": None})
        return out
    flops, byts = per[name]
    achieved = flops * steps_per_launch / avg_s
    peak = PEAK["f32" if esize == 4 else "f64"]
    out.update({
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": peak / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": stored_traffic(name, "fhn_n%d_%s" % (N, prec)),
        "forward_chunk": b1,
        "algorithmic_flops_per_launch": flops * steps_per_launch,
        "algorithmic_bytes_per_launch": byts * steps_per_launch,
        "achieved_GBps_algorithmic": byts * steps_per_launch / avg_s / 1e9,
        "hbm_frac_algorithmic": byts * steps_per_launch / avg_s / HBM_PEAK,
    })
    return out


def scan_kernel_table(prof, wl, prec):
    """Per step-level kernel: live average launch time, algorithmic GB/s and
    TFLOP/s, and their fractions of the HBM and vector peaks."""
    from paper_2310_01145_amd import costmodel

    esize = 4 if prec == "fp32" else 8
    per = costmodel.per_step(2, wl["q"], esize, costmodel.forward_chunk(wl["N"]))
    peak = PEAK["f32" if esize == 4 else "f64"]
    out = {}
    for name, (flops, byts) in per.items():
        if name not in prof:
            continue
        total_ms, launches = prof[name]
        avg_s = total_ms * 1e-3 / launches
        gbps = byts * wl["N"] / avg_s
        out[name] = {"avg_launch_us": avg_s * 1e6, "GBps": gbps / 1e9, "hbm_frac": gbps / HBM_PEAK,
                     "TFLOPs": flops * wl["N"] / avg_s / 1e12, "alu_frac": flops * wl["N"] / avg_s / peak,
                     "traffic_bytes_measured": stored_traffic(name, "fhn_n%d_%s" % (wl["N"], prec))}
    return out


def host_cpu():
    """(logical CPUs, CPU model) of the host the baseline runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_baseline(wl_full):
    """The CPU oracle (sequential FP64 square-root EKF/RTS IEKS, one thread)
    on the same workload: its own coarse-grid start, then Alg. 2 to
    Delta < 1e-10 (a few iterations)."""
    import oracle

    N = wl_full["N"]
    t = time.perf_counter()
    r = oracle.ieks(wl_full["field"], wl_full["params"], wl_full["y0"], wl_full["t0"], wl_full["t1"], wl_full["q"],
                    N, max_iter=20, tol=1e-10, want_cov=False, init="coarse")
    el = time.perf_counter() - t
    ncpu, model = host_cpu()
    return {"value": N * r["iterations"] / el, "unit": UNIT, "cores": 1, "kind": "oracle",
            "host_logical_cpus": ncpu, "host_cpu_model": model,
            "sample": "the whole FitzHugh-Nagumo solve (N=%d): the oracle's coarse-grid start and %d iterations to "
                      "Delta < 1e-10, FP64, single thread, %.1f s" % (N, r["iterations"], el)}


def mol_batch_run(pp, torch, prec, B=16, max_iter=20):
    """Method-of-lines batch (d=64, q=2, D=192, N=4096, B seeded instances)
    on the dense engine: one batched solve to convergence, every kernel timed
    by events (a few dozen launches per iteration, each milliseconds long)."""
    from paper_2310_01145_amd import costmodel, workloads

    sp, y0s = workloads.mol_batch(B=B)
    d, q, N = len(sp["y0"]), sp["q"], sp["N"]
    D = d * (q + 1)
    # warm-up: a short batch loads the kernels
    pp.solve_batch(sp["field"], sp["params"], y0s[:2], sp["t0"], sp["t1"], q, 64, precision=prec, fixed_iters=1)
    torch.cuda.synchronize()
    pp.profile_enable(True)
    t = time.perf_counter()
    r = pp.solve_batch(sp["field"], sp["params"], y0s, sp["t0"], sp["t1"], q, N, precision=prec, tol=1e-10,
                       max_iter=max_iter)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    prof = pp.profile_read()
    pp.profile_enable(False)
    its = r["iterations"]
    per = costmodel.dense_iteration_flops(D, d, q, N, 1)
    flops = {k: v * float(sum(its)) for k, v in per.items()}
    name = max(prof, key=lambda k: prof[k][0])
    peak = PEAK["f32" if prec == "fp32" else "f64"]
    kern = {}
    for k, (ms, n) in sorted(prof.items(), key=lambda kv: -kv[1][0]):
        kern[k] = {"total_ms": ms, "launches": n,
                   "TFLOPs": (flops[k] / (ms * 1e-3) / 1e12) if k in flops and ms > 0 else None}
    achieved = flops[name] / (prof[name][0] * 1e-3)
    total_flops = sum(flops.values())
    return r, {
        "value": N * float(sum(its)) / el,
        "ms_per_solve": 1e3 * el,
        "status": r["status"],
        "iterations": its,
        "roofline": {"kernel": name, "bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "avg_launch_us": prof[name][0] * 1e3 / prof[name][1], "launches": prof[name][1]},
        "whole_solve_TFLOPs": total_flops / el / 1e12,
        "whole_solve_frac": total_flops / el / peak,
        "kernels": kern,
    }


def mol_decoupled_run(pp, torch, prec, lin="diag_ek1", B=16, max_iter=400):
    """The same method-of-lines batch under an approximate Jacobian
    (DiagonalEK1 or EK0): the linearised model is block diagonal, so the solve
    runs as B x d decoupled problems of state size q+1 on the row-per-lane
    engine.  Timed to convergence (delta < 1e-10); the per-kernel table prices
    each step-level kernel by its algorithmic flops and bytes per chain step."""
    from paper_2310_01145_amd import costmodel, workloads

    sp, y0s = workloads.mol_batch(B=B)
    d, q, N = len(sp["y0"]), sp["q"], sp["N"]
    kw = dict(precision=prec, tol=1e-10, max_iter=max_iter, linearization=lin)
    pp.solve_batch(sp["field"], sp["params"], y0s[:2], sp["t0"], sp["t1"], q, 256, **kw)
    torch.cuda.synchronize()
    pp.profile_enable(True)
    t = time.perf_counter()
    r = pp.solve_batch(sp["field"], sp["params"], y0s, sp["t0"], sp["t1"], q, N, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    prof = pp.profile_read()
    pp.profile_enable(False)
    its = r["iterations"]
    esize = 4 if prec == "fp32" else 8
    per = costmodel.per_step(1, q, esize, costmodel.forward_chunk(N))
    chain_steps = float(d * N * sum(its))  # chain steps over all launches of a step-level kernel
    peak = PEAK["f32" if prec == "fp32" else "f64"]
    kern = {}
    for k, (ms, n) in sorted(prof.items(), key=lambda kv: -kv[1][0]):
        e = {"total_ms": ms, "launches": n}
        if k in per and ms > 0:
            fl, by = per[k]
            e.update({"TFLOPs": fl * chain_steps / (ms * 1e-3) / 1e12, "alu_frac": fl * chain_steps / (ms * 1e-3) / peak,
                      "GBps_algorithmic": by * chain_steps / (ms * 1e-3) / 1e9})
        kern[k] = e
    return r, {
        "value": N * float(sum(its)) / el,
        "ms_per_solve": 1e3 * el,
        "status": r["status"],
        "iterations": its,
        "chains": B * d,
        "kernels": kern,
    }


def _fhn_oracle_sample(N):
    """One whole oracle solve of the FitzHugh-Nagumo workload (worker of the
    per-core measurement); returns (time-steps x iterations, seconds)."""
    import oracle

    wl = workload(N, 0)
    t = time.perf_counter()
    r = oracle.ieks(wl["field"], wl["params"], wl["y0"], wl["t0"], wl["t1"], wl["q"], N, max_iter=20, tol=1e-10,
                    want_cov=False, init="coarse")
    return N * r["iterations"], time.perf_counter() - t


def _mol_oracle_sample(steps):
    """The method-of-lines oracle sample (worker of the per-core measurement)."""
    import oracle

    from paper_2310_01145_amd import workloads

    sp = workloads.mol(N=4096)
    t = time.perf_counter()
    r = oracle.ieks(sp["field"], sp["params"], sp["y0"], sp["t0"], sp["t1"] * steps / sp["N"], sp["q"], steps,
                    fixed_iters=2, want_cov=False)
    return steps * r["iterations"], time.perf_counter() - t


def per_core_instances(fn, arg, label):
    """One oracle instance per host core (at most 16, this host's share of a
    one-GPU node), all started together in fresh interpreters: the aggregate
    rate is the total work over the wall time until the last one ends."""
    import multiprocessing as mp

    ncpu, model = host_cpu()
    P = max(1, min(16, ncpu or 1))
    ctx = mp.get_context("spawn")
    t = time.perf_counter()
    with ctx.Pool(P) as pool:
        res = pool.map(fn, [arg] * P)
    wall = time.perf_counter() - t
    work = sum(w for w, _ in res)
    return {"value": work / wall, "unit": UNIT, "cores": P, "kind": "oracle", "instances": P,
            "host_logical_cpus": ncpu, "host_cpu_model": model,
            "sample": "%d concurrent oracle instances (one per core), each %s; wall %.1f s (slowest instance "
                      "%.1f s, interpreter start included)" % (P, label, wall, max(e for _, e in res))}


def mol_cpu_baseline(steps=96):
    """The oracle on a bounded sample of the method-of-lines workload: one
    instance, its first `steps` steps (same h), two iterations."""
    import oracle

    from paper_2310_01145_amd import workloads

    sp = workloads.mol(N=4096)
    t1 = sp["t1"] * steps / sp["N"]
    t = time.perf_counter()
    r = oracle.ieks(sp["field"], sp["params"], sp["y0"], sp["t0"], t1, sp["q"], steps, fixed_iters=2,
                    want_cov=False)
    el = time.perf_counter() - t
    ncpu, model = host_cpu()
    return {"value": steps * r["iterations"] / el, "unit": UNIT, "cores": 1, "kind": "oracle",
            "host_logical_cpus": ncpu, "host_cpu_model": model,
            "sample": "one method-of-lines instance (d=64, D=192), its first %d steps at the same h, 2 iterations, "
                      "FP64, single thread, %.1f s" % (steps, el)}


def copy_probe(torch, mib):
    """One plain device-to-device copy of mib MiB (read mib, write mib): the
    reference that scales the HBM byte counters of a profiling run."""
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=1 << 18)
    ap.add_argument("--iters", type=int, default=0, help="fixed iterations per solve (0: to Delta < 1e-10)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-lorenz", action="store_true", help="skip the Lorenz-63 (D=15) measurement")
    ap.add_argument("--no-constant-start", action="store_true", help="skip the constant-start report")
    ap.add_argument("--no-extras", action="store_true", help="skip the logistic latency and the N sweep")
    ap.add_argument("--no-mol", action="store_true", help="skip the method-of-lines batch (dense engine, D=192)")
    ap.add_argument("--no-mol-fp64", action="store_true", help="method-of-lines batch in FP32 only")
    ap.add_argument("--no-stream", action="store_true", help="skip the served stream (4096 requests)")
    ap.add_argument("--stream-requests", type=int, default=4096)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain copy of this many MiB first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); the path is a single-GPU solver and no "
              "multi-GPU figure is produced.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2310_01145_amd as pp

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    pp.load_library()
    if args.copy_probe_mib > 0:
        copy_probe(torch, args.copy_probe_mib)

    wl = workload(args.N, args.iters)
    print("bench: workload FHN N=%d iters=%d" % (wl["N"], wl["iters"]), file=sys.stderr, flush=True)
    # every solve computes its own coarse-grid start inside the timed region
    r32 = run_gpu(pp, torch, wl, "fp32", args.steps, args.warmup, not args.no_profile)
    print("bench: fp32 done %.3f ms/solve" % r32["ms_per_step"], file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        r64 = run_gpu(pp, torch, wl, "fp64", args.steps, args.warmup, False)
        print("bench: fp64 done %.3f ms/solve" % r64["ms_per_step"], file=sys.stderr, flush=True)
    # the same solve with 20 fixed iterations (the per-iteration rate with the start amortised)
    f20 = run_gpu(pp, torch, workload(args.N, 20), "fp32", max(2, args.steps // 2), 1, False)
    print("bench: fp32 20 iterations done %.3f ms/solve" % f20["ms_per_step"], file=sys.stderr, flush=True)
    from paper_2310_01145_amd import costmodel

    coarse_m = costmodel.coarse_points(wl["N"])
    line = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "FitzHugh-Nagumo a=b=0.2 c=3, y0=(-1,1), t in [0,100], IWP(3) D=8, N=%d, one whole "
                               "solve: coarse-grid start then IEKS iterations to Delta < 1e-10 (at most 20)" % wl["N"],
                   "N": wl["N"], "q": wl["q"], "d": 2, "precision": "fp32_sqrt",
                   "initial_trajectory": "the library's coarse-grid start (sequential EKS on %d coarse steps of %d "
                                         "fine steps, bridged by the prior), computed inside every timed solve"
                                         % (coarse_m, -(-wl["N"] // coarse_m))},
        "latency_ms_p50": r32["latency_ms_p50"],
        "latency_ms_p99": r32["latency_ms_p99"],
        "iterations_per_solve": r32["iterations_per_solve"][0],
        "solve_status": r32["status"][0],
        "start": r32["start"],
        "fixed_20_iterations_fp32": {"value": f20["value"], "ms_per_step": f20["ms_per_step"],
                                     "status": f20["status"][0]},
    }
    if not args.no_constant_start:
        line["constant_start"] = {"fp32": constant_start(pp, wl, "fp32")}
        if not args.no_fp64:
            line["constant_start"]["fp64"] = constant_start(pp, wl, "fp64")
    if r64 is not None:
        line["fp64"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                        "latency_ms_p50": r64["latency_ms_p50"], "latency_ms_p99": r64["latency_ms_p99"],
                        "iterations_per_solve": r64["iterations_per_solve"][0], "solve_status": r64["status"][0],
                        "start": r64["start"]}
    if r32["profile"]:
        # the dominant kernel, timed by events inside the timed region
        line["roofline"] = roofline(r32["profile"], wl, "fp32", r32["profile_untimed"])
        # the dominant kernel of the iterations (the scans' step-level kernels)
        it = {k: v for k, v in r32["profile_untimed"].items() if not k.startswith("coarse")}
        line["roofline_iteration"] = roofline(it, wl, "fp32", r32["profile_untimed"])
        # every kernel, from the untimed profiled solve before it
        line["scan_kernels"] = scan_kernel_table(r32["profile_untimed"], wl, "fp32")
        line["kernel_ms_per_solve"] = {k: v[0] for k, v in sorted(r32["profile_untimed"].items(),
                                                                  key=lambda kv: -kv[1][0])}
    if not args.no_lorenz:
        # chaos caps the reachable Delta near 1e-8 in FP64 (rounding grows like
        # exp(0.9 t)), so the Lorenz solves run 20 fixed iterations
        lw = lorenz_workload(args.N, 20)
        cold = pp.solve(lw["field"], lw["params"], lw["y0"], lw["t0"], lw["t1"], lw["q"], lw["N"], precision="fp32",
                        max_iter=3)
        l32 = run_gpu(pp, torch, lw, "fp32", args.steps, args.warmup, False, d=3)
        l64 = run_gpu(pp, torch, lw, "fp64", max(1, args.steps // 2), 1, False, d=3)
        print("bench: lorenz done %.3f / %.3f ms/solve" % (l32["ms_per_step"], l64["ms_per_step"]), file=sys.stderr,
              flush=True)
        line["lorenz"] = {
            "workload": "Lorenz-63 s=10 r=28 b=8/3, y0=(1,1,1), t in [0,20], IWP(4) D=15, N=%d, coarse-grid start "
                        "then %d IEKS iterations (the constant start diverges)" % (lw["N"], lw["iters"]),
            "value_fp32": l32["value"], "ms_per_step_fp32": l32["ms_per_step"],
            "value_fp64": l64["value"], "ms_per_step_fp64": l64["ms_per_step"],
            "status_fp32": l32["status"][0], "status_fp64": l64["status"][0],
            "iterations_fp32": l32["iterations_per_solve"][0], "iterations_fp64": l64["iterations_per_solve"][0],
            "constant_start_fp32": {"status": cold["status"], "iterations": cold["iterations"],
                                    "final_delta": cold["final_delta"]},
        }
    if not args.no_extras:
        line["logistic_c0"] = logistic_latency(pp, torch)
        line["fhn_n_sweep"] = n_sweep(pp, torch, args.iters)
        line["fhn_n1048576_scan_kernels"] = beyond_cache(pp, torch)
        print("bench: extras done", file=sys.stderr, flush=True)
    if not args.no_mol:
        m32r, m32 = mol_batch_run(pp, torch, "fp32")
        print("bench: mol fp32 done %.1f ms/solve" % m32["ms_per_solve"], file=sys.stderr, flush=True)
        line["mol_batch"] = {
            "workload": "method of lines u_t = 0.01 u_xx + u(1-u), d=64 periodic points, IWP(2) D=192, N=4096, "
                        "t in [0,1], 16 seeded initial profiles in one batched solve, constant start, "
                        "to tol 1e-10 (at most 20 iterations)",
            "fp32": m32,
        }
        if not args.no_mol_fp64:
            m64r, m64 = mol_batch_run(pp, torch, "fp64")
            print("bench: mol fp64 done %.1f ms/solve" % m64["ms_per_solve"], file=sys.stderr, flush=True)
            a = m32r["mean"][:, :, ::3].double()
            b = m64r["mean"][:, :, ::3]
            line["mol_batch"]["fp64"] = m64
            line["mol_batch"]["fp32_vs_fp64_e0_relerr"] = float((a - b).abs().max() / b.abs().max())
            del m64r, a, b
        # DiagonalEK1 on the same batch: decoupled chains, cost linear in d
        g32r, g32 = mol_decoupled_run(pp, torch, "fp32")
        print("bench: mol diag_ek1 fp32 done %.1f ms/solve" % g32["ms_per_solve"], file=sys.stderr, flush=True)
        g64r, g64 = mol_decoupled_run(pp, torch, "fp64")
        print("bench: mol diag_ek1 fp64 done %.1f ms/solve" % g64["ms_per_solve"], file=sys.stderr, flush=True)
        a = g32r["mean"][:, :, ::3].double()
        b = g64r["mean"][:, :, ::3]
        dg = {"workload": "the same batch under DiagonalEK1 (F_y ~ diag F_y): 1024 decoupled chains of state "
                          "size 3, constant start, to tol 1e-10 (at most 400 iterations)",
              "fp32": g32, "fp64": g64, "fp32_vs_fp64_e0_relerr": float((a - b).abs().max() / b.abs().max()),
              "time_to_solution_vs_ek1_fp32": m32["ms_per_solve"] / g32["ms_per_solve"]}
        c = m32r["mean"][:, :, ::3].double()
        # both fixed points solve the ODE at the grid points; they differ by
        # about the discretisation error
        dg["fixed_point_vs_ek1_e0_relerr"] = float((b - c).abs().max() / c.abs().max())
        line["mol_batch"]["diag_ek1"] = dg
        del m32r, g32r, g64r, a, b, c
        if not args.no_cpu_baseline:
            line["mol_batch"]["cpu_baseline"] = mol_cpu_baseline()
            line["mol_batch"]["cpu_baseline_per_core"] = per_core_instances(
                _mol_oracle_sample, 96, "the method-of-lines sample above (96 steps, 2 iterations)")
    if not args.no_stream:
        from paper_2310_01145_amd import serve

        st = serve.run(n_requests=args.stream_requests, load=0.8)
        print("bench: served stream done", file=sys.stderr, flush=True)
        line["served_stream"] = st
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl)
        line["cpu_baseline_per_core"] = per_core_instances(
            _fhn_oracle_sample, wl["N"], "the whole FitzHugh-Nagumo solve above")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
