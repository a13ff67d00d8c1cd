"""Benchmark: neighbour-pair updates per second of the relaxation step on one MI355X.

One "step" is a full relaxation step of the hot path (half drift, F -> stress -> T, pairwise force
and kick, the swept pairwise damping on the steps the random-choice rule picks, second half drift
and the FP64 reductions).  The headline workload is the largest single-GPU body: a 3D column
0.2 x 0.2 x 1.0 m at dp = 0.001 m (200 x 200 x 1000 free particles plus 4 clamped base layers,
40,160,000 particles, 3,178,450,616 CSR entries), h = 1.3 dp, neo-Hookean E = 5e6 Pa, nu = 0.3,
lateral body force 5 m/s^2, alpha = 0.2.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  value = (CSR entries) x (steps) / (wall time of the timed steps), FP32 forces,
stress and damping with FP64 displacement and reductions; the same body in plain FP64 is timed
beside it, and so is the 1.26M-particle 3D cantilever.  The line also carries the roofline of the
kernel that takes most of the step (the method's algorithmic bytes per launch over its measured mean
launch time), the FP64 oracle timed on the host cores (serial and shared-memory mode), and the
serving measurement: the first 8 requests of the serving stream through the FP32 request server
(capacity, solves/s, time to the 1e-4 residual) against the plain one-at-a-time FP64 path.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PASSES = ("drift", "passA", "passB", "passD", "passC", "finish")


def algorithmic_bytes(dim: int, precision: int, n: int, nnz: int, ncolour_launches: int) -> dict:
    """Bytes the method itself must move per launch of each pass (each array the pass needs read or
    written once, neighbour re-reads taken to hit on-chip caches).  FP32 3D figures, per CSR entry
    and per particle:
      pass A  4 B per entry (the neighbour index) + 130 B per particle
      pass B  4 B per entry + 140 B per particle
      pass C  40 B per particle
      pass D  a forward (or backward) sweep of the K colour launches reads every entry's index and
              every velocity once and writes the velocities once: 4 B per entry + 24 B per particle
              per sweep, (4 nnz + 24 n) / K per colour launch
    Other precisions and dimensions scale each per-particle figure by the sizes of the arrays it
    stands for (A: u, v, X0, B0 in, T, u_h out; B: X0, T, v in, v out, row offsets; C: u_h, v in,
    u out; D: v in and out)."""
    R = 4 if precision == 32 else 8
    D = dim
    K = max(1, ncolour_launches)
    # per-particle terms: exact FP32 3D values of the method's byte model, scaled to other precisions
    # and dimensions by the array sizes they stand for
    a_pp = 130.0 * (8 * D + R * D + 8 * D + 2 * R * D * D + 8 * D) / (8 * 3 + 4 * 3 + 8 * 3 + 2 * 4 * 9 + 8 * 3)
    b_pp = 140.0 * (8 * D + R * D * D + 2 * R * D + 8) / (8 * 3 + 4 * 9 + 2 * 4 * 3 + 8)
    c_pp = 40.0 * (8 * D + R * D + 8 * D) / (8 * 3 + 4 * 3 + 8 * 3)
    d_pp = 2.0 * R * D
    return {
        "passA": 4 * nnz + a_pp * n,
        "passB": 4 * nnz + b_pp * n,
        "passC": c_pp * n,
        "passD": (4 * nnz + d_pp * n) / K,
        "finish": 0,
        "drift": 0,
    }


def design_bytes(dim: int, precision: int, n: int, nnz: int, has_accel: bool, ncolour_launches: int) -> dict:
    """Bytes this implementation's data structures move per launch (reported beside the method's
    algorithmic bytes): every per-particle array a pass touches once, every CSR entry's 2-byte
    LDS slot (plus its 4/8-byte damping factor in pass D); pass D stages the velocities of every
    cell's 3^D-cell neighbourhood and writes them back, and over a colour's cells these
    neighbourhoods cover the whole body, so v moves twice per colour launch."""
    R = 4 if precision == 32 else 8
    D = dim
    K = max(1, ncolour_launches)
    return {
        "passA": n * (8 + 8 * D + 8 * D + R * D + 1 + R * D * D + R * D * D + 8 * D) + 2 * nnz,
        "passB": n * (8 + 8 * D + R * D * D + 2 * R * D + 1 + (R * D if has_accel else 0)) + 2 * nnz,
        "passC": n * (8 * D + R * D + 1 + 8 * D),
        "passD": n * 2 * R * D + (nnz * (2 + R) + n * 8) // K,
        "finish": 0,
        "drift": 0,
    }


KERNEL_SOURCES = ("setup.hip", "step.hip", "damp.hip", "bricks.hpp", "internal.hpp", "devmath.hpp")


def kernel_sources_sha256() -> str:
    """Hash of the kernel sources' code: comments and whitespace are dropped, so a comment edit does
    not invalidate counters taken from the same code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2103_08932_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(workload: str, precision: int) -> dict:
    """HBM bytes per launch of each pass from the committed rocprofv3 counter summary of this
    workload (FETCH_SIZE and WRITE_SIZE, scaled by the factors a plain copy kernel gives), or {} when
    there is none or the kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_fp{precision}.txt")
    if not os.path.exists(path):
        return {}
    sha, out = None, {}
    for line in open(path):
        f = line.split()
        if len(f) == 2 and f[0] == "sha256":
            sha = f[1]
        elif len(f) == 3 and f[0] == "traffic":
            out[f[1]] = int(f[2])
    return out if sha == kernel_sources_sha256() else {}


def make_workload(name: str):
    import workloads
    if name == "c2":
        return workloads.c2_cantilever_3d()
    if name == "c2_small":
        return workloads.c2_cantilever_3d(nx=100, ny=20, nz=20)
    if name == "c2_coarse":
        # the same 1.0 x 0.1 x 0.1 m beam at dp = 0.004 (156k particles)
        return workloads.c2_cantilever_3d(nx=250, ny=25, nz=25, dp=0.004)
    if name == "twist":
        return workloads.twisting_cantilever_3d()
    if name == "c3":
        return workloads.c3_block()
    if name == "c5":
        return workloads.c5_column()
    if name == "c5_sample":
        # the column's construction, dp, material and load at 60 x 60 x 40 free particles
        return workloads.c5_column(nx=60, ny=60, nz=40)
    if name == "c1":
        return workloads.c1_cantilever_2d()
    raise SystemExit(f"unknown workload {name}")


def host_cpu() -> dict:
    """The host's processor model, logical CPU count and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable": usable}


def cpu_baseline(sample_wb, alpha: float, log=print, max_threads: int = 16) -> dict:
    """The FP64 oracle on the host cores, setup excluded: 5 plain and 5 forced-damped steps of
    `sample_wb`, combined as the cost of a random-choice step, plain + alpha (damped - plain), once
    single-threaded and once in the oracle's shared-memory mode on the usable cores (at most
    max_threads; the mode is bit-identical to the serial oracle)."""
    import oracle
    cpu = host_cpu()
    threads_all = max(1, min(max_threads, cpu["usable"] or 1))
    runs = {}
    for th in sorted({1, threads_all}):
        got = oracle.set_threads(th)
        t0 = time.perf_counter()
        ob = oracle.OracleBody(sample_wb)
        setup = time.perf_counter() - t0
        nnz = ob.nnz
        t0 = time.perf_counter()
        ob.step(5, force=0)
        t_plain = (time.perf_counter() - t0) / 5
        t0 = time.perf_counter()
        ob.step(5, force=1)
        t_damped = (time.perf_counter() - t0) / 5
        ob.close()
        per_step = t_plain + alpha * (t_damped - t_plain)
        runs[got] = {"value": nnz / per_step, "s_per_plain_step": t_plain, "s_per_damped_step": t_damped,
                     "setup_s": setup}
        log(f"[cpu] oracle, {got} thread(s): plain {t_plain:.3f} s, damped {t_damped:.3f} s per step, "
            f"{nnz / per_step:.3e} pair updates/s")
    oracle.set_threads(1)
    best = max(runs)
    return {"value": runs[best]["value"], "unit": "pair updates/s", "cores": best, "kind": "oracle",
            "sample": f"{sample_wb.name} ({sample_wb.n} particles, {nnz} CSR entries; the headline body's "
                      f"construction, dp, material and load at a size the oracle steps in seconds): 5 plain + "
                      f"5 forced-damped steps, combined as plain + alpha (damped - plain), alpha = {alpha}, "
                      "setup excluded",
            "single_thread_value": runs[1]["value"], "runs": {str(k): v for k, v in runs.items()},
            "host": cpu}


def small_relax_vs_oracle(wb, log=print) -> dict:
    """The 2D cantilever (1,040 particles) relaxed to its own tolerance (1e-6, at most 10,000 steps) by
    the FP64 oracle on one thread and by the plain FP64 GPU path: wall time, steps, pair updates/s.
    A body this small leaves the GPU latency-bound (about 20 launches per step)."""
    import oracle
    import paper_2103_08932_amd as tl
    import torch
    out = {"workload": wb.name, "particles": wb.n, "tol": wb.tol, "max_steps": wb.max_steps}
    oracle.set_threads(1)
    ob = oracle.OracleBody(wb)
    t0 = time.perf_counter()
    rep = ob.relax(wb.tol, wb.max_steps)
    wall = time.perf_counter() - t0
    out["oracle_1_thread"] = {"steps": rep["steps"], "seconds": wall, "converged": rep["converged"],
                              "residual": rep["residual"], "pair_updates_per_s": ob.nnz * rep["steps"] / wall}
    ob.close()
    b = tl.from_workload(wb, precision=64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = b.relax_until(wb.tol, wb.max_steps)
    wall = time.perf_counter() - t0
    nnz = b.body_info()[1]
    b.close()
    out["gpu_fp64"] = {"steps": rep["steps"], "seconds": wall, "converged": bool(rep["converged"]),
                       "residual": rep["residual"], "pair_updates_per_s": nnz * rep["steps"] / wall}
    log(f"[cpu] {wb.name} to {wb.tol:g}: oracle {out['oracle_1_thread']['steps']} steps in "
        f"{out['oracle_1_thread']['seconds']:.2f} s, GPU FP64 {out['gpu_fp64']['steps']} steps in {wall:.2f} s")
    return out


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x, dtype=float), q)) if len(x) else None


def _wait_all(srv, tickets, log):
    reps = []
    t0 = time.perf_counter()
    for t in tickets:
        rep = None
        waits = 0
        while rep is None:
            rep = srv.wait(t, 5.0)
            waits += 1
            if rep is None and waits % 6 == 0:
                log(f"[serve]   waiting for ticket {t} ({len(reps)} of {len(tickets)} done, "
                    f"{time.perf_counter() - t0:.0f} s)")
        reps.append(rep)
        what = f"{rep['steps']} steps, residual {rep['residual']:.2e}" if rep["status"] >= 0 else rep.get("error")
        log(f"[serve]   ticket {t}: status {rep['status']}, {what}")
    return reps


def serving(M: int, budget_gb: float, slots: int, rate_factor: float = 0.8, seed: int = 2, log=print,
            fp64: bool = True, rate: float = 0.0) -> dict:
    """Requests 0 .. M-1 of the serving stream (seed 2): half 2D, half 3D cantilevers / plates of
    5k-500k particles, each relaxed to its own 1e-4 residual.
      1. FP32 server, all requests submitted at once: capacity C = M / makespan.
      2. FP32 server, Poisson arrivals at rate_factor * C: solves/s and latency (arrival -> result).
      3. The plain one-at-a-time FP64 path (create, relax_until, get_displacement per request): its
         service times give FIFO latencies for the same arrivals.
    Also the relative L2 error of every FP32 result against the FP64 result of the same request.
    With fp64=False only steps 1 and 2 run (serving_fp64 covers step 3 in a process of its own); with
    rate > 0 step 1 is skipped and the arrivals come at that rate (requests per second)."""
    import threading

    import numpy as np
    import paper_2103_08932_amd as tl
    import workloads

    reqs = [workloads.serving_request(r, seed=seed) for r in range(M)]
    budget = int(budget_gb * (1 << 30))
    log(f"[serve] {M} requests, particles {sum(w.n for w in reqs)} total "
        f"({min(w.n for w in reqs)}..{max(w.n for w in reqs)}), {sum(w.dim == 2 for w in reqs)} 2D")

    # 1. closed loop
    if rate > 0:
        reps32, u32, closed_lat, st_closed, makespan = None, None, [], {"peak_active": None, "pool_peak": None}, None
    else:
        with tl.Server(budget, max_slots=slots, precision=tl.FP32) as srv:
            t0 = time.perf_counter()
            tickets = [srv.submit(w) for w in reqs]
            reps32 = _wait_all(srv, tickets, log)
            makespan = time.perf_counter() - t0
            u32 = [srv.result(t) if r["status"] >= 0 else None for t, r in zip(tickets, reps32)]
            closed_lat = [float(srv.times(t)[3] - srv.times(t)[0]) for t, r in zip(tickets, reps32) if r["converged"]]
            st_closed = srv.stats()
        cap = M / makespan
        log(f"[serve] closed loop: makespan {makespan:.2f} s, capacity {cap:.3f} requests/s, "
            f"{sum(bool(r['converged']) for r in reps32)} of {M} converged")
        # 2. open loop at rate_factor * capacity
        rate = rate_factor * cap
    arr = workloads.arrival_times(M, rate, seed)
    with tl.Server(budget, max_slots=slots, precision=tl.FP32) as srv:
        tickets = [None] * M
        start = time.perf_counter()

        def feeder():
            for k, w in enumerate(reqs):
                delay = start + arr[k] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets[k] = srv.submit(w)
                log(f"[serve]   submitted request {k} at {time.perf_counter() - start:.1f} s")

        th = threading.Thread(target=feeder)
        th.start()
        th.join()
        reps_open = _wait_all(srv, tickets, log)
        tm = np.array([srv.times(t) for t in tickets])
        st_open = srv.stats()
    ok_open = np.array([bool(r["converged"]) for r in reps_open])
    if reps32 is None:      # no closed loop: the open loop's reports stand for the requests' outcomes
        reps32 = reps_open
    ok32 = [bool(r["converged"]) for r in reps32]
    lat32 = (tm[:, 3] - tm[:, 0])[ok_open]
    span32 = tm[:, 3].max() - tm[:, 0].min()
    log(f"[serve] open loop at {rate:.3f} req/s: p50 {_pct(lat32, 50):.2f} s, p99 {_pct(lat32, 99):.2f} s")

    fp32_part = {"converged": int(sum(ok32)), "failed": int(sum(r["status"] < 0 for r in reps32)),
                 "step_limited": int(sum(r["status"] == 1 for r in reps32)),
                 "latency_completions": int(ok_open.sum()), "status": [r["status"] for r in reps32],
                 "capacity_solves_per_s": sum(ok32) / makespan if makespan else None, "closed_loop_makespan_s": makespan,
                 "closed_loop_p50_s": _pct(closed_lat, 50), "closed_loop_p99_s": _pct(closed_lat, 99),
                 "arrival_rate_per_s": rate, "solves_per_s": int(ok_open.sum()) / span32,
                 "p50_latency_s": _pct(lat32, 50), "p99_latency_s": _pct(lat32, 99),
                 "latency_s": [float(x) for x in (tm[:, 3] - tm[:, 0])],
                 "steps": [r["steps"] for r in reps32],
                 "peak_active": st_open["peak_active"], "peak_active_closed": st_closed["peak_active"],
                 "pool_peak_bytes": st_closed["pool_peak"], "budget_bytes": budget, "slots": slots}
    if not fp64:
        return {"requests": M, "workload": f"serving stream requests 0..{M - 1} (seed {seed})",
                "particles": [w.n for w in reqs], "dims": [w.dim for w in reqs], "fp32_batched": fp32_part}
    # 3. sequential plain FP64
    service, steps64, nnz, err, ok64 = [], [], [], [], []
    for k, w in enumerate(reqs):
        t1 = time.perf_counter()
        b = tl.from_workload(w, precision=tl.FP64)
        nnz.append(b.body_info()[1])
        try:
            rep = b.relax_until(w.tol, w.max_steps)
            u64 = b.get_displacement()
            ok64.append(bool(rep["converged"]))
            steps64.append(rep["steps"])
        except tl.TLSPHError as e:
            u64 = None
            ok64.append(False)
            steps64.append(None)
            log(f"[serve]   fp64 request {k}: {e}")
        b.close()
        service.append(time.perf_counter() - t1)
        if u64 is not None and u32[k] is not None and ok32[k] and ok64[-1]:
            err.append(float(np.linalg.norm(u32[k] - u64) / max(np.linalg.norm(u64), 1e-300)))
            log(f"[serve]   fp64 request {k}: {steps64[-1]} steps in {service[-1]:.2f} s, fp32 error {err[-1]:.2e}")
    finish, lat64 = 0.0, []
    for k in range(M):
        finish = max(arr[k], finish) + service[k]
        if ok64[k]:
            lat64.append(finish - arr[k])
    span64 = finish - arr[0]
    pairs32 = sum(n * r["steps"] for n, r in zip(nnz, reps32))
    return {
        "requests": M, "workload": f"serving stream requests 0..{M - 1} (seed {seed})",
        "particles": [w.n for w in reqs], "dims": [w.dim for w in reqs],
        "note": "solves/s counts requests that reached the 1e-4 residual; latency percentiles are over those "
                "requests; a request that fails (J <= 0 under extreme deflection) fails the same way in FP64",
        "fp32_batched": {"converged": int(sum(ok32)), "failed": int(sum(r["status"] < 0 for r in reps32)),
                         "step_limited": int(sum(r["status"] == 1 for r in reps32)),
                         "latency_completions": int(ok_open.sum()), "status": [r["status"] for r in reps32],
                         "capacity_solves_per_s": sum(ok32) / makespan if makespan else None, "closed_loop_makespan_s": makespan,
                         "closed_loop_p50_s": _pct(closed_lat, 50), "closed_loop_p99_s": _pct(closed_lat, 99),
                         "arrival_rate_per_s": rate, "solves_per_s": int(ok_open.sum()) / span32,
                         "p50_latency_s": _pct(lat32, 50), "p99_latency_s": _pct(lat32, 99),
                         "steps": [r["steps"] for r in reps32], "pair_updates_per_s": pairs32 / makespan if makespan else None,
                         "peak_active": st_open["peak_active"], "peak_active_closed": st_closed["peak_active"],
                         "pool_peak_bytes": st_closed["pool_peak"], "budget_bytes": budget, "slots": slots},
        "fp64_sequential": {"converged": int(sum(ok64)), "not_converged": int(len(ok64) - sum(ok64)),
                            "latency_completions": len(lat64), "capacity_solves_per_s": sum(ok64) / sum(service),
                            "solves_per_s": sum(ok64) / span64,
                            "p50_latency_s": _pct(lat64, 50), "p99_latency_s": _pct(lat64, 99),
                            "service_s": service, "steps": steps64},
        "fp32_vs_fp64_rel_l2": {"max": max(err) if err else None, "median": _pct(err, 50), "count": len(err)},
        "speedup_capacity": (sum(ok32) / makespan) / max(sum(ok64) / sum(service), 1e-300),
    }


def serving_fp64(ids, seed: int = 2, log=print, error: bool = True) -> dict:
    """The plain one-at-a-time FP64 path on requests `ids` of the serving stream (create, relax_until,
    get_displacement per request; its wall time is the request's service time), and, untimed, the
    same request through the single-body FP32 path (bit-identical to its served result) for the
    FP32-vs-FP64 error.  FIFO latencies need the service times of every earlier request, so they are
    computed where the ranges are joined.  error=False skips the FP32 rerun (no error figure)."""
    import numpy as np
    import paper_2103_08932_amd as tl
    import workloads
    out = {"ids": list(ids), "service_s": [], "status": [], "steps": [], "fp32_steps": [], "fp32_status": [],
           "rel_l2_fp32_vs_fp64": []}
    for r in ids:
        w = workloads.serving_request(r, seed=seed)
        res = {}
        for prec in ((64, 32) if error else (64,)):
            t1 = time.perf_counter()
            b = tl.from_workload(w, precision=prec)
            try:
                rep = b.relax_until(w.tol, w.max_steps)
                res[prec] = (rep["status"], rep["steps"], b.get_displacement())
            except tl.TLSPHError as e:
                res[prec] = (e.code, None, None)
            b.close()
            if prec == 64:
                out["service_s"].append(time.perf_counter() - t1)
        res.setdefault(32, (None, None, None))
        out["status"].append(res[64][0])
        out["steps"].append(res[64][1])
        out["fp32_status"].append(res[32][0])
        out["fp32_steps"].append(res[32][1])
        u64, u32 = res[64][2], res[32][2]
        ok = res[64][0] == 0 and res[32][0] == 0
        out["rel_l2_fp32_vs_fp64"].append(float(np.linalg.norm(u32 - u64) / max(np.linalg.norm(u64), 1e-300))
                                          if ok else None)
        log(f"[serve64] request {r} ({w.dim}D, {w.n} particles): fp64 status {res[64][0]} {res[64][1]} steps in "
            f"{out['service_s'][-1]:.2f} s; fp32 status {res[32][0]} {res[32][1]} steps; "
            f"error {out['rel_l2_fp32_vs_fp64'][-1]}")
    return out


def relax(wb, precision: int, tol: float, max_steps: int, chunk: int = 5000, log=print, keep_u=None,
          snap_at: int = 0, snap=None) -> dict:
    """Time to the residual tol: relax_until in chunks of `chunk` steps (the residual tracking carries
    over between calls, so this equals one call), setup excluded.  keep_u (a list) receives the final
    displacement.  With snap_at > 0 the chunks also stop exactly at step snap_at and `snap` (a list)
    receives the displacement there; a run that stops earlier is stepped on to snap_at after its
    timing ends."""
    import paper_2103_08932_amd as tl
    import torch
    t0 = time.perf_counter()
    b = tl.from_workload(wb, precision=precision)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    n, nnz, _, W = b.body_info()
    steps, damped, status = 0, 0, "not converged"
    rep = None
    t0 = time.perf_counter()
    try:
        while steps < max_steps:
            lim = min(chunk, max_steps - steps)
            if steps < snap_at:
                lim = min(lim, snap_at - steps)
            rep = b.relax_until(tol, lim)
            steps += rep["steps"]
            damped += rep["damped_steps"]
            log(f"[relax] fp{precision} step {steps} residual {rep['residual']:.3e} E_k {rep['kinetic_energy']:.3e} "
                f"t {time.perf_counter() - t0:.1f} s")
            if steps == snap_at and snap is not None:
                snap.append(b.get_displacement())
            if rep["converged"]:
                status = "converged"
                break
    except tl.TLSPHError as e:
        status = f"failed: {e}"
    wall = time.perf_counter() - t0
    extra = {}
    if not status.startswith("failed"):
        u = b.get_displacement()
        if keep_u is not None:
            keep_u.append(u)
        p = tip_probe(wb)
        extra = {"probe_u": [float(x) for x in u[p]], "max_abs_u": float(abs(u).max()),
                 "force_residual": rep["force_residual"] if rep else None}
        try:
            vm = b.get_von_mises()
            extra["von_mises_max_pa"] = float(vm.max())
        except tl.TLSPHError as e:
            extra["von_mises_max_pa"] = f"failed: {e}"
        if snap is not None and 0 < snap_at and steps < snap_at:
            b.step(snap_at - steps)
            snap.append(b.get_displacement())
    b.close()
    return {"precision": f"fp{precision}", "status": status, "steps": steps, "damped_steps": damped, "window": W,
            "seconds": wall, "setup_s": setup, "residual": rep["residual"] if rep else None,
            "pair_updates_per_s": nnz * steps / wall if wall > 0 else None, "particles": n, "pairs": nnz, **extra}


def tip_probe(wb) -> int:
    """Input index of the probe S of Sec. 4.1: the free particle at the beam's free end (largest x)
    nearest to the cross-section's centre line."""
    import numpy as np
    X = wb.X0
    free = np.flatnonzero(wb.clamped == 0)
    xmax = X[free, 0].max()
    end = free[X[free, 0] > xmax - 0.5 * wb.dp]
    c = X[free, 1:].min(axis=0) + 0.5 * (X[free, 1:].max(axis=0) - X[free, 1:].min(axis=0))
    return int(end[np.argmin(((X[end, 1:] - c) ** 2).sum(axis=1))])


def damping_study(names, precision: int = 32, tol: float = 1e-4, log=print, seconds_per_run: float = 45.0,
                  schemes=("pairwise", "particle")) -> dict:
    """The paper's damping-parameter study (Sec. 4.1) on synthetic bodies: random choice alpha in
    {1, 0.2} x artificial viscosity eta in {1, 5, 10} eta0 x both damping schemes.  eta0 is Eq. 36
    with the paper's beta = d / l (thickness over length) and L = d, so 10 eta0 is the workloads'
    default beta = 1.  Each run relaxes to `tol` (or stops at its step or wall-time budget, or on
    divergence) and records the probe's displacement history and the time to the residual; each run
    is also printed as one JSON line when it ends."""
    import numpy as np
    import paper_2103_08932_amd as tl
    import torch
    out = []
    for name in names:
        base = make_workload(name)
        Xf = base.X0[base.clamped == 0]
        ext = Xf.max(axis=0) - Xf.min(axis=0) + base.dp
        beta0 = float(min(ext[1:]) / ext[0])
        probe = tip_probe(base)
        comp = base.dim - 1 if base.dim == 2 else 1        # the deflection component (y)
        chunk, budget = (500, 100_000) if base.dim == 2 else (2000, 160_000)
        ref_u = None
        for scheme in schemes:
            for alpha in (1.0, 0.2):
                for mult in (1, 5, 10):
                    wb = make_workload(name)
                    wb.scheme, wb.alpha, wb.beta = scheme, alpha, beta0 * mult
                    log(f"[study] {wb.name} {scheme} alpha {alpha} eta {mult} eta0")
                    b = tl.from_workload(wb, precision=precision)
                    torch.cuda.synchronize()
                    hist, steps, damped, status, rep = [], 0, 0, "not converged", None
                    t0 = time.perf_counter()
                    try:
                        while steps < budget and time.perf_counter() - t0 < seconds_per_run:
                            rep = b.relax_until(tol, min(chunk, budget - steps))
                            steps += rep["steps"]
                            damped += rep["damped_steps"]
                            u = b.get_displacement()
                            hist.append((steps, float(u[probe, comp])))
                            if rep["converged"]:
                                status = "converged"
                                break
                    except tl.TLSPHError as e:
                        status = f"failed: {e}"
                    wall = time.perf_counter() - t0
                    u_end = b.get_displacement() if status == "converged" else None
                    b.close()
                    if scheme == "pairwise" and alpha == 0.2 and mult == 10 and u_end is not None:
                        ref_u = u_end
                    keep = hist[:: max(1, len(hist) // 40)]
                    out.append({"workload": wb.name, "scheme": scheme, "alpha": alpha, "eta_over_eta0": mult,
                                "status": status, "steps": steps, "damped_steps": damped, "seconds": wall,
                                "dt_s": rep["dt"] if rep else None, "residual": rep["residual"] if rep else None,
                                "probe_final": hist[-1][1] if hist else None, "probe_history": keep,
                                "_u": u_end})
                    log(f"[study]   {status}, {steps} steps in {wall:.1f} s, probe {out[-1]['probe_final']}")
                    print(json.dumps({"damping_study_run": {k: v for k, v in out[-1].items() if k != "_u"}}),
                          flush=True)
        for r in out:
            if r["workload"] == base.name:
                u = r.pop("_u")
                r["rel_l2_vs_pairwise_alpha0.2_10eta0"] = (
                    float(np.linalg.norm(u - ref_u) / np.linalg.norm(ref_u))
                    if (u is not None and ref_u is not None) else None)
    return {"tol": tol, "precision": f"fp{precision}", "runs": out}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--extra-workloads", default="c2", help="comma-separated workloads also timed in FP32 and FP64")
    ap.add_argument("--no-fp64", action="store_true", help="do not time the workload in plain FP64 as well")
    ap.add_argument("--cpu-sample", default="c5_sample", help="workload the oracle is timed on")
    ap.add_argument("--scheme", default="pairwise", choices=("pairwise", "particle"),
                    help="damping split: pairwise (Sec. 3.2) or particle-by-particle (Sec. 3.1)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pass-timing", action="store_true", help="do not record per-pass HIP events")
    ap.add_argument("--serving", type=int, default=8, metavar="M",
                    help="also serve the first M requests of the serving stream (0 = skip)")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving measurement")
    ap.add_argument("--serving-rate", type=float, default=0.0,
                    help="with --serving-only: skip the closed loop and send the arrivals at this rate (requests/s)")
    ap.add_argument("--serving-no-fp64", action="store_true",
                    help="with --serving-only: only the FP32 server phases (closed and open loop)")
    ap.add_argument("--serving-fp64-ids", default="", metavar="A:B",
                    help="only the sequential plain FP64 path (and the FP32 error) on requests A .. B-1")
    ap.add_argument("--serving-fp64-no-error", action="store_true",
                    help="with --serving-fp64-ids: time the FP64 path only, without the FP32 rerun for the error")
    ap.add_argument("--serving-budget-gb", type=float, default=16.0)
    ap.add_argument("--serving-slots", type=int, default=32)
    ap.add_argument("--relax", default="", metavar="PRECISIONS",
                    help="only measure the time to the workload's 1e-4 residual, e.g. 32 or 32,64")
    ap.add_argument("--relax-max-steps", type=int, default=400000)
    ap.add_argument("--relax-tol", type=float, default=1e-4,
                    help="residual of --relax (a tiny value with a step limit compares precisions at equal steps)")
    ap.add_argument("--damping-study", default="", metavar="WORKLOADS",
                    help="comma-separated workloads for the alpha x eta x scheme study (e.g. c1,c2_coarse)")
    ap.add_argument("--study-schemes", default="pairwise,particle")
    ap.add_argument("--study-seconds", type=float, default=45.0, help="wall-time budget of one study run")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device copy of GIB GiB (5 times): the reference kernel for scaling "
                         "the HBM traffic counters")
    ap.add_argument("--force-damping", type=int, default=-1, choices=(-1, 0, 1),
                    help="-1: random choice (the method); 1: damp every timed step (profiling the damping pass)")
    ap.add_argument("--timing-steps", type=int, default=200,
                    help="steps of the second, per-pass-timed region (HIP events around every launch)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the multi-GPU slab decomposition is a design, not code)", file=sys.stderr)
        return 2

    import torch
    import paper_2103_08932_amd as tl

    torch.cuda.set_device(0)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    if args.copy_calibration > 0:
        nbytes = int(args.copy_calibration * (1 << 30))
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": nbytes, "launches": 5}), flush=True)
        return 0
    if args.relax:
        import numpy as np
        wb = make_workload(args.workload)
        wb.scheme = args.scheme
        us, snap = [], []
        precs = [int(p) for p in args.relax.split(",")]
        out = [relax(wb, precs[0], args.relax_tol, args.relax_max_steps, log=log, keep_u=us)]
        for p in precs[1:]:
            # the later runs also keep their state at the first run's stopping step
            out.append(relax(wb, p, args.relax_tol, args.relax_max_steps, log=log, keep_u=us,
                             snap_at=out[0]["steps"] if us else 0, snap=snap))
        res = {"workload": wb.name, "scheme": wb.scheme, "tol": args.relax_tol, "max_steps": args.relax_max_steps,
               "runs": out}
        if len(us) == 2 and len(out) == 2:
            # the two end states (each at its own stopping step, or both at the step limit), relative L2
            # of the difference
            res["rel_l2_u_first_vs_second"] = float(np.linalg.norm(us[0] - us[1]) / np.linalg.norm(us[1]))
        if snap and us:
            # the two precisions at the same step count (the first run's stopping step)
            res["rel_l2_u_equal_steps"] = float(np.linalg.norm(us[0] - snap[0]) / np.linalg.norm(snap[0]))
            res["equal_steps"] = out[0]["steps"]
        print(json.dumps({"time_to_residual": res}), flush=True)
        return 0
    if args.damping_study:
        print(json.dumps({"damping_study": damping_study(args.damping_study.split(","), args.precision, log=log,
                                                         seconds_per_run=args.study_seconds,
                                                         schemes=tuple(args.study_schemes.split(",")))}), flush=True)
        return 0
    if args.serving_fp64_ids:
        a, b = (int(x) for x in args.serving_fp64_ids.split(":"))
        print(json.dumps({"serving_fp64": serving_fp64(range(a, b), log=log,
                                                       error=not args.serving_fp64_no_error)}), flush=True)
        return 0
    if args.serving_only:
        print(json.dumps({"serving": serving(max(1, args.serving), args.serving_budget_gb, args.serving_slots,
                                             log=log, fp64=not args.serving_no_fp64,
                                             rate=args.serving_rate)}), flush=True)
        return 0
    log(f"[bench] host: {host_cpu()}")
    wb = make_workload(args.workload)
    wb.scheme = args.scheme
    head = throughput(wb, args.precision, args.steps, args.warmup, 0 if args.no_pass_timing else args.timing_steps,
                      log=log, force=args.force_damping)
    passes, roof, step_hbm = {}, None, None
    if head["prof"]:
        K = 27 if wb.dim == 3 else 9
        ab = algorithmic_bytes(wb.dim, args.precision, head["n"], head["nnz"], K)
        db = design_bytes(wb.dim, args.precision, head["n"], head["nnz"], wb.accel is not None, K)
        # the stored counters are those of the pairwise damping kernel
        traffic = measured_traffic(wb.name, args.precision) if wb.scheme == "pairwise" else {}
        moved = 0.0
        for name in PASSES:
            ms, cnt = head["prof"].get(name, (0.0, 0))
            if cnt:
                us = 1e3 * ms / cnt
                passes[name] = {"ms_total": ms, "launches": cnt, "us_per_launch": us,
                                "algorithmic_bytes": ab[name],
                                "gbs": ab[name] / (us * 1e-6) / 1e9 if ms > 0 and ab[name] else None,
                                "design_bytes": db[name], "traffic_bytes": traffic.get(name)}
                moved += ab[name] * cnt
        # the roofline of the kernel that takes most of the step
        dom = max((k for k in passes if ab[k] > 0), key=lambda k: passes[k]["ms_total"])
        ach = passes[dom]["gbs"]
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": traffic.get(dom),
                "algorithmic_bytes_per_launch": ab[dom], "us_per_launch": passes[dom]["us_per_launch"],
                "design_bytes_per_launch": db[dom]}
        # the whole step: the method's bytes of every launch of the timing region over its kernel time
        ktime = sum(v["ms_total"] for v in passes.values()) * 1e-3
        step_hbm = {"algorithmic_bytes_per_step": moved / head["timing_steps"],
                    "gbs_kernel_time": moved / ktime / 1e9, "frac_kernel_time": moved / ktime / 1e9 / HBM_PEAK_GBS,
                    "gbs_wall": moved / head["timing_steps"] / (head["ms_per_step"] * 1e-3) / 1e9}
    line = {
        "metric": "pair updates/s",
        "value": head["value"],
        "unit": "pair updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": wb.name, "particles": head["n"], "pairs": head["nnz"], "dim": wb.dim,
                   "alpha": wb.alpha, "scheme": wb.scheme, "damped_steps": head["damped_steps"],
                   "setup_s": head["setup_s"],
                   "precision": f"fp{args.precision} stress/force/damping, fp64 displacement and reductions"
                   if args.precision == 32 else "fp64 throughout"},
        "roofline": roof,
        "step_hbm": step_hbm,
        "passes": passes,
    }
    if args.precision == 32 and not args.no_fp64:
        f64 = throughput(wb, 64, args.steps, args.warmup, 0, log=log)
        line["fp64"] = {"value": f64["value"], "ms_per_step": f64["ms_per_step"], "damped_steps": f64["damped_steps"],
                        "setup_s": f64["setup_s"], "fp32_speedup": head["value"] / f64["value"]}
    if args.extra_workloads:
        line["extra"] = {}
        for name in args.extra_workloads.split(","):
            ew = make_workload(name)
            ew.scheme = args.scheme
            r32 = throughput(ew, 32, args.steps, args.warmup, 0, log=log)
            r64 = throughput(ew, 64, args.steps, args.warmup, 0, log=log)
            line["extra"][name] = {"workload": ew.name, "particles": r32["n"], "pairs": r32["nnz"],
                                   "fp32": {k: r32[k] for k in ("value", "ms_per_step", "damped_steps")},
                                   "fp64": {k: r64[k] for k in ("value", "ms_per_step", "damped_steps")}}
    del wb
    if args.serving > 0:
        try:
            line["serving"] = serving(args.serving, args.serving_budget_gb, args.serving_slots, log=log)
        except Exception as e:  # reported in the line; the step measurement above stands
            line["serving"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        sample = make_workload(args.cpu_sample)
        line["cpu_baseline"] = cpu_baseline(sample, sample.alpha, log=log)
        line["cpu_baseline"]["c1_to_convergence"] = small_relax_vs_oracle(make_workload("c1"), log=log)
    print(json.dumps(line), flush=True)
    return 0


def throughput(wb, precision: int, steps: int, warmup: int, timing_steps: int, log=print, force: int = -1) -> dict:
    """Creates the body (setup timed on its own), runs `warmup` untimed steps, then times `steps`
    random-choice steps between two device synchronisations.  With timing_steps > 0 a second region
    records HIP events around every launch on the body's stream for the per-pass times (kept out of
    the timed region: the events add launch overhead)."""
    import paper_2103_08932_amd as tl
    import torch
    log(f"[bench] workload {wb.name}: {wb.n} particles, fp{precision}, {wb.scheme} damping")
    t0 = time.perf_counter()
    body = tl.from_workload(wb, precision=precision)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    n, nnz, _, _ = body.body_info()
    log(f"[bench] setup {setup_s:.2f} s, nnz {nnz}")
    if warmup:
        body.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = body.step(steps, force)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[bench] fp{precision}: {steps} steps ({rep['damped_steps']} damped) in {elapsed:.3f} s, "
        f"{nnz * steps / elapsed:.3e} pair updates/s")
    prof = {}
    if timing_steps > 0:
        body.profile(True)
        body.step(timing_steps)
        prof = body.profile_read()
        body.profile(False)
    body.close()
    return {"value": nnz * steps / elapsed, "ms_per_step": 1e3 * elapsed / steps, "damped_steps": rep["damped_steps"],
            "setup_s": setup_s, "n": n, "nnz": nnz, "prof": prof, "timing_steps": timing_steps}


if __name__ == "__main__":
    sys.exit(main())
