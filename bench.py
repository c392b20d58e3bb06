#!/usr/bin/env python3
"""Benchmark of the preconditioned Krylov hot path on one MI355X.

Workload (the metric's configuration): block-Jacobi PCG on the IPM normal
equations M = A D A^T + 1e-8 I with A 200,000 x 500,000 (8 N(0,1) nonzeros per
column, localized pattern), 20 dense columns at 30% density kept as a
low-rank operator term, D log-uniform in [1e-6, 1e6], 64 contiguous blocks,
GEOMEAN filter tau = 1e-3 with the dropped magnitude added to the diagonal,
ILU(0) per block, tolerance 1e-8 on the true relative residual.

The dense columns are also eliminated as a border of the preconditioner, and
ILU(0) breakdowns are handled by the shifted refactorisation policy.

A step is one complete solve (x0 = 0 to relres <= 1e-8) of that system with
its inputs resident in HBM; the preconditioner is built once before timing.
Both the plain FP64 PCG and the FP32-inner / FP64-refined form are timed; the
line reports the faster as `value` and both under `modes`.  Beside it: the
oracle on one thread and on the host cores, measured copy and read ceilings,
and the SpMV / block-Jacobi launch times on the full-size C4 system (5.2M
rows, 256 blocks), whose working set is far larger than the Infinity Cache.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s to rel. residual 1e-8; achieved HBM GB/s; p50/p99 solve latency"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def percentile(xs, q):
    s = sorted(xs)
    if not s:
        return None
    k = (len(s) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def build_c5(req):
    """One request of the served stream (run in a worker process)."""
    from ipm_inputs import gen
    return gen.c5_system(req)


def build_c4():
    """The first system of the C4 sequence at full size (worker process)."""
    from ipm_inputs import gen
    return gen.IPMSequence(steps=30).system(0)


def run_mode(sd, torch, system, opts, steps, warmup, tol, solve_log=None):
    t0 = time.time()
    solver = sd.from_system(system, opts)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    b = torch.as_tensor(system.b, device="cuda:0")
    x = torch.empty_like(b)
    log(f"  setup {setup_s:.2f} s")
    for w in range(warmup):
        _, its, rr, st = solver.solve(b, x, tol)
        log(f"  warmup {w}: status {st} iterations {its} relres {rr:.2e}")
    lat, its_all, rr_all = [], [], []
    spmv_ms = bj_ms = 0.0
    spmv_n = bj_n = 0
    info = None
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(steps):
        t1 = time.perf_counter()
        _, its, rr, st = solver.solve(b, x, tol, log=solve_log, extra={"config": system.name, "step": k})
        lat.append((time.perf_counter() - t1) * 1e3)
        its_all.append(its)
        rr_all.append(rr)
        info = solver.info()
        p = 1 if opts.precision == sd.FP32_IR else 0
        spmv_ms += info["spmv_ms"][0] + info["spmv_ms"][1]
        spmv_n += info["spmv_launches"][0] + info["spmv_launches"][1]
        bj_ms += info["bj_ms"][0] + info["bj_ms"][1]
        bj_n += info["bj_launches"][0] + info["bj_launches"][1]
        log(f"  step {k}: status {st} iterations {its} (outer {info['outer_iters']}, fp64 fallbacks "
            f"{info['fp64_fallbacks']}) relres {rr:.2e} {lat[-1]:.1f} ms")
        if st != sd.OK:
            raise RuntimeError(f"solve failed with status {st}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    # true residual of the last solution, compensated FP64 (library kernel)
    _, nr = solver.residual(b, x)
    relres = nr / float(torch.linalg.vector_norm(b).item())
    p = 1 if opts.precision == sd.FP32_IR else 0
    # algorithmic bytes of the whole solve: every Krylov iteration moves
    # bytes_per_iter (SpMV + fused PCG/block-Jacobi step + direction update)
    solve_bytes = float(np.mean(its_all)) * info["bytes_per_iter"]
    res = dict(solves_per_s=steps / total, ms_per_solve=1e3 * total / steps, iterations=its_all,
               solve_gbps=solve_bytes / (total / steps) / 1e9, bytes_per_iter=info["bytes_per_iter"],
               relres=relres, setup_s=setup_s, p50_ms=percentile(lat, 0.5), p99_ms=percentile(lat, 0.99),
               outer=info["outer_iters"], fallbacks=info["fp64_fallbacks"], restarts=info["restarts"],
               nnz_kept=info["nnz_kept"], shifted_blocks=info["shifted_blocks"], max_shift=info["max_shift"],
               spmv_launches=spmv_n, bj_launches=bj_n,
               spmv_avg_us=1e3 * spmv_ms / max(spmv_n, 1), bj_avg_us=1e3 * bj_ms / max(bj_n, 1),
               spmv_bytes=info["spmv_bytes"][p], bj_bytes=info["bj_bytes"][p],
               spmv_bytes_fp64=info["spmv_bytes"][0], spmv_bytes_fp32=info["spmv_bytes"][1])
    if spmv_n:
        # which precision's SpMV dominates the launches
        res["spmv_gbps"] = res["spmv_bytes"] / (res["spmv_avg_us"] * 1e-6) / 1e9
        res["bj_gbps"] = res["bj_bytes"] / (res["bj_avg_us"] * 1e-6) / 1e9
    solver.close()
    return res


def run_serving(sd, torch, gen, systems, active, modes, solve_log=None):
    """Served C5 stream: the first len(systems) requests of the seeded
    stream (built before timing), solved to 1e-8 with the C2 filter in each
    of `modes`, by the serving loop with shared launches (one stream, one
    launch per kernel per iteration of all running requests, HIP-graph
    replay) and continuous batching up to `active` requests.  Per mode all
    requests arrive at t = 0 (saturated: the service rate mu); the first
    mode is run again with Poisson arrivals at 0.8 mu.  Latency = arrival to
    completion (queueing, setup and solve)."""
    from paper_2604_23979_amd.serve import Request, Server
    count = len(systems)

    def progress(tag):
        def done(req):
            k = done.count = getattr(done, "count", 0) + 1
            if k % 10 == 0 or k == count:
                log(f"    {tag}: {k}/{count} requests done")
        return done
    prec = {"fp64": sd.FP64, "fp32ir": sd.FP32_IR}
    out = {"workload": f"C5: first {count} requests of the seeded stream (rows log-uniform 1e4..5e5, 6-10 per "
                       f"column, D spread 1e8, 8-128 blocks; {sum(s.n for s in systems)} rows in all), "
                       f"GEOMEAN tau=1e-3 + DROPSUM, PCG to 1e-8; served with shared launches, up to {active} "
                       f"requests at once",
           "requests": count, "closed_loop": {}}
    for mode in modes:
        o = sd.Options(precision=prec[mode], filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM,
                       pivot=sd.PIVOT_SHIFT, shift0=1e-2, max_iter=60_000, refine_delta=0.3)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()   # each leg starts from the same free HBM
        srv = Server(options=o, max_active=active, on_done=progress(f"closed loop {mode}"), log=solve_log)
        srv.run([Request(s, 0.0, i) for i, s in enumerate(systems)])
        st = srv.stats()
        st["iterations"] = int(sum(r.iters for r in srv.done))
        out["closed_loop"][mode] = st
        log(f"  closed loop {mode}: {st}")
        if mode == modes[0]:
            mu = st["solves_per_s"]
            arr = gen.poisson_arrivals(count, 0.8 * mu)
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            srv2 = Server(options=o, max_active=active, on_done=progress(f"Poisson {mode}"), log=solve_log)
            srv2.run([Request(s, float(arr[i]), i) for i, s in enumerate(systems)])
            out["poisson_0.8mu"] = dict(srv2.stats(), mode=mode, rate_per_s=0.8 * mu)
            log(f"  Poisson at 0.8 mu ({mode}): {out['poisson_0.8mu']}")
    # the plain FP64 GPU solve: one request at a time, setup + solve on one
    # stream, no overlap
    o64 = sd.Options(precision=sd.FP64, filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM,
                     pivot=sd.PIVOT_SHIFT, shift0=1e-2, max_iter=60_000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, its_tot, ok = [], 0, 0
    for s in systems:
        b = torch.as_tensor(s.b, device="cuda:0")
        sv = sd.from_system(s, o64)
        _, its, _, st = sv.solve(b, tol=1e-8)
        torch.cuda.synchronize()
        sv.close()
        lat.append(1e3 * (time.perf_counter() - t0))
        its_tot += its
        ok += st == sd.OK
        if len(lat) % 10 == 0:
            log(f"    plain FP64: {len(lat)}/{count} requests done")
    span = time.perf_counter() - t0
    out["plain_fp64"] = dict(requests=count, ok=ok, makespan_s=round(span, 3), solves_per_s=round(count / span, 4),
                             p50_ms=round(float(np.percentile(lat, 50)), 1),
                             p99_ms=round(float(np.percentile(lat, 99)), 1), iterations=its_tot)
    log(f"  plain FP64, one at a time: {out['plain_fp64']}")
    served = out["closed_loop"].get("fp32ir")
    if served:
        out["served_fp32ir_over_plain_fp64"] = round(served["solves_per_s"] / out["plain_fp64"]["solves_per_s"], 3)
    out["all_ok"] = all(v["ok"] == count for v in out["closed_loop"].values()) and ok == count
    return out


def run_c1(sd, torch, gen, steps):
    """C1: the small system (2,000 rows, 4 blocks, ILU(0) without filter, FP64
    PCG).  Its working set sits in the caches, so it is latency- and
    launch-bound: reported as ms per solve and us per iteration."""
    s = gen.c1()
    sv = sd.from_system(s, sd.Options())
    b = torch.as_tensor(s.b, device="cuda:0")
    sv.solve(b, tol=1e-8)  # warm-up
    times, its, rr = [], 0, 1.0
    for _ in range(max(1, steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, its, rr, st = sv.solve(b, tol=1e-8)
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0))
    sv.close()
    ms = float(np.median(times))
    out = dict(workload="C1: A 2,000x5,000, 5 N(0,1) per column, D log-uniform [1e-4,1e4], 4 blocks, ILU(0), "
                        "FP64 PCG", n=s.n, nnz=s.nnz, iterations=its, relres=rr, ms_per_solve=round(ms, 3),
               us_per_iteration=round(1e3 * ms / max(its, 1), 2), solves_per_s=round(1e3 / ms, 2))
    log(f"  C1: {out}")
    return out


def run_bbd(sd, torch, gen, steps):
    """C3: BBD-preconditioned GMRES(30) on the 1.5M-row bordered system (32
    blocks of 46,750 rows, 4,096-row border); setup (ILU(0) of the blocks, the
    dense Schur complement on MFMA and its LU) is timed apart from the
    solves; the relative residual is the library's own compensated FP64
    one (the oracle checks the residual kernel in the tests)."""
    t0 = time.time()
    s = gen.c3(1.0)
    log(f"  C3: n={s.n} nnz={s.nnz} border={s.n_border} blocks={s.nblocks} built in {time.time() - t0:.1f} s")
    o = sd.Options(method=sd.BBD, krylov=sd.GMRES, restart=30, spd=False, max_iter=10_000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sv = sd.from_system(s, o)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t1
    b = torch.as_tensor(s.b, device="cuda:0")
    times, its = [], []
    x = None
    for _ in range(max(1, steps)):
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        x, it, rr, st = sv.solve(b, tol=1e-8)
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t2))
        its.append(it)
        log(f"  C3 solve: status {st}, {it} GMRES iterations, relres {rr:.2e}, {times[-1]:.1f} ms")
    true_rr = rr
    sv.close()
    out = dict(workload="C3: 32 x 46,750 banded-random blocks + 4,096 border, GMRES(30), BBD, FP64 dense Schur",
               n=s.n, nnz=s.nnz, border=s.n_border, setup_s=round(setup_s, 3), iterations=its,
               ms_per_solve=round(float(np.median(times)), 2), solves_per_s=round(1e3 / float(np.median(times)), 3),
               relres=true_rr)
    log(f"  C3: {out}")
    return out


def run_ipm_sequence(sd, torch, gen, steps, rows, policy="fixed", precision="fp32ir"):
    """IPM sequence (C4): `steps` consecutive systems A D_k A^T + 1e-8 I on
    one pattern, blocks of ~20k rows, GEOMEAN 1e-3 + DROPSUM PCG; the
    preconditioner is refactored every 5 systems and reused (new operator
    values only) in between.  policy "adaptive" also ends a reuse period on
    convergence degradation (a reused solve capped at 1.5x the iterations of
    the last fresh one is refactored and solved again).  The relative
    residual of every system is the library's own compensated FP64 one."""
    from paper_2604_23979_amd.ipm import SequenceSolver
    t0 = time.time()
    nblocks = max(1, int(round(rows / 20_312)))   # the full-size block height (5.2M rows / 256 blocks)
    q = gen.IPMSequence(m=rows, nblocks=nblocks, steps=max(steps, 2),
                        progress=lambda msg: log(f"  IPM sequence: {msg}"))
    log(f"  IPM sequence: n={rows} nnz={q.col.shape[0]} built in {time.time() - t0:.1f} s")
    prec = {"fp64": sd.FP64, "fp32ir": sd.FP32_IR}[precision]
    o = sd.Options(precision=prec, filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM,
                   pivot=sd.PIVOT_SHIFT, shift0=1e-2, max_iter=60_000, refine_delta=0.3)
    seq = SequenceSolver(lambda system, opts: sd.from_system(system, opts), o, reuse_every=5,
                         degrade=1.5 if policy == "adaptive" else float("inf"))
    recs = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for k in range(steps):
        sk = q.system(k)
        vals = torch.as_tensor(sk.val, device="cuda:0")
        b = torch.as_tensor(sk.b, device="cuda:0")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, rec = seq.step(k, sk, vals, b, tol=1e-8)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        true_rr = rec.relres
        recs.append(dict(k=k, kind=rec.kind, ms=round(1e3 * (t2 - t1), 1), iterations=rec.iterations,
                         status=rec.status, relres=true_rr))
        log(f"  system {k} ({rec.kind}): {rec.iterations} its, {1e3 * (t2 - t1):.0f} ms, "
            f"status {rec.status}, relres {true_rr:.2e}")
    total = time.perf_counter() - t_all
    seq.close()
    gpu_s = sum(r["ms"] for r in recs) / 1e3
    return {"workload": f"C4: {steps} systems, n={rows}, {nblocks} blocks of ~20k rows, refactor every 5, "
                        f"policy {policy}, {precision}",
            "systems": recs,
            "gpu_seconds": round(gpu_s, 3), "wall_seconds_incl_host_checks": round(total, 1),
            "systems_per_s": round(steps / gpu_s, 4),
            "all_converged": all(r["status"] == sd.OK and r["relres"] <= 1e-8 for r in recs)}


def measured_traffic(which, mode):
    """HBM bytes per launch from the committed counter summary of this kernel
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None when the
    summary is missing or the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_k_{which}_c2_{mode}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec.get("sources", []):
        with open(os.path.join(ROOT, src), "rb") as g:
            h.update(g.read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(system, gpu_iters, seconds, opts_o, threads):
    """The oracle (plain C; OpenMP only over independent rows and blocks) on
    a bounded sample of the same solve: the preconditioner build, then a
    fixed number of PCG iterations on `threads` threads, scaled to solves/s
    with the FP64 iteration count measured on the GPU."""
    import oracle as O
    O.set_threads(threads)
    try:
        t0 = time.perf_counter()
        P = O.BJ(system, **opts_o)
        setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.pcg_bj(system, P, tol=1e-30, maxit=3)
        per = (time.perf_counter() - t0) / 3
        k = max(3, int(seconds / max(per, 1e-6)))
        t0 = time.perf_counter()
        O.pcg_bj(system, P, tol=1e-30, maxit=k)
        t_iter = (time.perf_counter() - t0) / k
    finally:
        O.set_threads(1)
    solve_s = t_iter * gpu_iters
    return {"value": round(1.0 / solve_s, 6), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} FP64 PCG iterations of the full system ({t_iter * 1e3:.2f} ms each on {threads} "
                      f"thread(s)) scaled by the {gpu_iters} iterations of one GPU FP64 solve; preconditioner "
                      f"build {setup:.2f} s excluded like on the GPU"}


def copy_ceiling(torch, nbytes=1 << 30, reps=20):
    """Measured bandwidth ceilings on this GPU: a plain device copy and a
    device-wide read (sum) of `nbytes`, timed with events."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    bb = torch.empty_like(a)
    for _ in range(3):
        bb.copy_(a)
        a.sum()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bb.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy = 2 * nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    e0.record()
    for _ in range(reps):
        a.sum()
    e1.record()
    torch.cuda.synchronize()
    read = nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del a, bb
    torch.cuda.empty_cache()
    return {"copy_gbps": round(copy, 1), "read_gbps": round(read, 1), "bytes": nbytes,
            "kind": "torch copy_ and sum of a 1 GiB FP64 buffer, HIP events"}


def host_cpu():
    """CPU model and the cores this process may use (capped at the 16 of
    one GPU's host share)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return model, avail, max(1, min(16, avail))


def run_c4_kernels(sd, torch, s, iters):
    """C4 at its full size (5.2M rows, 256 blocks, the first system of the
    IPM sequence): the per-iteration cost and the SpMV and block-Jacobi
    launch times on a working set far larger than the 256 MB Infinity Cache.
    Only `iters` PCG iterations are run (HIP events on every launch): at this
    size ILU(0) block Jacobi needs more than 10^4 iterations per system, so
    complete solves do not fit the benchmark (the true residual after the
    iterations is reported)."""
    log(f"  C4: n={s.n} nnz={s.nnz} blocks={s.nblocks}")
    b = torch.as_tensor(s.b, device="cuda:0")
    out = {"workload": "C4 system 0 at full size: A 5,200,000 x 8,320,000, 4 N(0,1)/col localized, D spread 1e2, "
                       "256 blocks, GEOMEAN tau=1e-3 + DROPSUM, SHIFT 1e-2, ILU(0), PCG; "
                       f"{iters} iterations timed per mode, not a complete solve",
           "n": s.n, "nnz": s.nnz, "nblocks": s.nblocks}
    for name, prec in (("fp64", sd.FP64), ("fp32ir", sd.FP32_IR)):
        o = sd.Options(precision=prec, filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM,
                       pivot=sd.PIVOT_SHIFT, shift0=1e-2, max_iter=iters, kernel_timing=1, refine_every=10 ** 9)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sv = sd.from_system(s, o)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t1
        sv.solve(b, tol=1e-8)  # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, its, rr, st = sv.solve(b, tol=1e-8)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        inf = sv.info()
        p = 1 if prec == sd.FP32_IR else 0
        sp_us = 1e3 * inf["spmv_ms"][p] / max(1, inf["spmv_launches"][p])
        bj_us = 1e3 * inf["bj_ms"][p] / max(1, inf["bj_launches"][p])
        out[name] = {"setup_s": round(setup, 3), "iterations": its, "relres_after": rr,
                     "ms_per_iteration": round(1e3 * dt / max(its, 1), 4), "nnz_kept": inf["nnz_kept"],
                     "shifted_blocks": inf["shifted_blocks"],
                     "spmv_us": round(sp_us, 2), "spmv_bytes": inf["spmv_bytes"][p],
                     "spmv_gbps": round(inf["spmv_bytes"][p] / (sp_us * 1e-6) / 1e9, 1),
                     "bj_us": round(bj_us, 2), "bj_bytes": inf["bj_bytes"][p],
                     "bj_gbps": round(inf["bj_bytes"][p] / (bj_us * 1e-6) / 1e9, 1)}
        log(f"  C4 {name}: {out[name]}")
        sv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workload (tests only)")
    ap.add_argument("--modes", default="fp64,fp32ir")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing", type=int, default=64,
                    help="HIP-event timing of the SpMV and block-Jacobi launches of every k-th iteration inside the "
                         "timed solves (0: off)")
    ap.add_argument("--max-iter", type=int, default=60_000)
    ap.add_argument("--refine-delta", type=float, default=0.3)
    ap.add_argument("--profile-iters", type=int, default=0,
                    help="profiling run: only this many iterations per mode, no JSON line")
    ap.add_argument("--extra-steps", type=int, default=3,
                    help="timed solves of the modes after the first (one warm-up each)")
    ap.add_argument("--serve", type=int, default=48,
                    help="served C5 requests (closed loop, then Poisson at 0.8x that rate; 0: skip)")
    ap.add_argument("--serve-active", type=int, default=32)
    ap.add_argument("--serve-modes", default="fp32ir,fp64",
                    help="precisions of the served stream (the first also gets the Poisson run)")
    ap.add_argument("--log", default=None,
                    help="append one JSON record per solve (C2 solves and served requests) to this JSONL file")
    ap.add_argument("--gen-workers", type=int, default=8,
                    help="processes that build the C4 and C5 inputs while the GPU runs C2 (0: build them in this "
                         "process, after C2)")
    ap.add_argument("--c4", type=int, default=0,
                    help="also run the IPM sequence (this many systems, refactor every 5) at --c4-rows rows")
    ap.add_argument("--c4-rows", type=int, default=520_000)
    ap.add_argument("--c4-policy", default="fixed", choices=["fixed", "adaptive"],
                    help="fixed: refactor every 5 systems; adaptive: also on convergence degradation")
    ap.add_argument("--c4-precision", default="fp32ir", choices=["fp32ir", "fp64"])
    ap.add_argument("--c1", type=int, default=0, help="also time this many solves of the small system C1")
    ap.add_argument("--c3", type=int, default=0,
                    help="also run the BBD / GMRES(30) system C3 (setup, then this many solves)")
    ap.add_argument("--c4-kernels", type=int, default=300,
                    help="PCG iterations timed on the full-size C4 system (0: skip; also run by --profile-iters)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="profiling run: first copy a buffer of this many bytes three times (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"the solver runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the whole workload runs on one MI355X)", file=sys.stderr)
        sys.exit(2)

    # the C4 and C5 inputs are built by worker processes (started here,
    # before this process touches the GPU) while the GPU runs C2
    from concurrent.futures import ProcessPoolExecutor
    from ipm_inputs import gen
    pool = fut_c4 = None
    fut_c5 = []
    want_c4 = args.c4_kernels > 0 and args.scale == 1.0 and args.profile_iters == 0
    want_c5 = args.serve > 0 and args.profile_iters == 0
    if (want_c4 or want_c5) and args.gen_workers > 0:
        pool = ProcessPoolExecutor(max_workers=args.gen_workers)
        if want_c4:
            fut_c4 = pool.submit(build_c4)
        if want_c5:
            fut_c5 = [pool.submit(build_c5, r) for r in gen.c5_requests()[:args.serve]]

    import torch
    import paper_2604_23979_amd as sd

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    if args.copy_bytes > 0:
        # a plain device copy of known size; its FETCH_SIZE / WRITE_SIZE
        # counters scale those of the solver kernels to bytes
        src = torch.empty(args.copy_bytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.copy_bytes} bytes three times")
        del src, dst
    t0 = time.time()
    log("generating the workload ...")
    system = gen.c2(args.scale)
    log(f"  {system.name}: n={system.n} nnz={system.nnz} blocks={system.nblocks} "
        f"low-rank k={system.lowrank[0].shape[1]} nnz_U={system.lowrank[0].nnz} ({time.time() - t0:.1f} s)")
    common = dict(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM, pivot=sd.PIVOT_SHIFT,
                  shift0=1e-2, kernel_timing=args.timing, max_iter=args.max_iter,
                  refine_delta=args.refine_delta, border=True)
    if args.profile_iters > 0:
        b_dev = torch.as_tensor(system.b, device="cuda:0")
        for m in args.modes.split(","):
            prec = {"fp64": sd.FP64, "fp32ir": sd.FP32_IR, "fp32restart": sd.FP32_IR_RESTART}[m]
            o = sd.Options(precision=prec, **dict(common, max_iter=args.profile_iters))
            sv = sd.from_system(system, o)
            _, its, rr, st = sv.solve(b_dev, torch.empty_like(b_dev), 1e-8)
            torch.cuda.synchronize()
            log(f"profile {m}: {its} iterations, status {st}, relres {rr:.2e}")
            sv.close()
        if args.c4_kernels > 0 and args.scale == 1.0:
            run_c4_kernels(sd, torch, build_c4(), args.c4_kernels)
        if args.c1 > 0:
            run_c1(sd, torch, gen, args.c1)
        if args.c3 > 0:
            run_bbd(sd, torch, gen, args.c3)
        return
    solve_log = None
    if args.log:
        from paper_2604_23979_amd.solvelog import JsonlLog
        solve_log = JsonlLog(args.log)
    modes = {}
    mode_list = args.modes.split(",")
    for i, m in enumerate(mode_list):
        prec = {"fp64": sd.FP64, "fp32ir": sd.FP32_IR, "fp32restart": sd.FP32_IR_RESTART}[m]
        steps, warmup = (args.steps, args.warmup) if i == 0 else (args.extra_steps, 1)
        log(f"mode {m} ({steps} timed solves{', the JSON value' if i == 0 else ''}):")
        modes[m] = run_mode(sd, torch, system, sd.Options(precision=prec, **common), steps, warmup, 1e-8, solve_log)
        modes[m]["timed_solves"] = steps
        log(f"  {m}: {modes[m]['solves_per_s']:.3f} solves/s, SpMV {modes[m].get('spmv_gbps', 0):.0f} GB/s, "
            f"BJ {modes[m].get('bj_gbps', 0):.0f} GB/s")
    # the value is the first mode's: the one timed over exactly --steps solves
    best = mode_list[0]
    r = modes[best]
    fp64_its = modes["fp64"]["iterations"][-1] if "fp64" in modes else r["iterations"][-1]
    # roofline of the dominant kernel (the larger share of the solve time
    # between the SpMV and the fused block-Jacobi step): algorithmic bytes of
    # one launch over its average duration from HIP events inside the solves
    roof = None
    if r.get("spmv_gbps"):
        sp_t = r["spmv_avg_us"]
        bj_t = r["bj_avg_us"]
        which = "bj" if bj_t > sp_t else "spmv"
        prec = "FP64" if best == "fp64" else "FP32"
        name = {"bj": f"k_bj ({prec})", "spmv": f"k_spmv ({prec})"}[which]
        gbps = r[f"{which}_gbps"]
        roof = {"bound": "hbm", "kernel": name, "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(gbps / HBM_PEAK_GBPS, 4),
                "traffic": measured_traffic(which, best),
                "bytes_per_launch": r[f"{which}_bytes"], "avg_launch_us": round(r[f"{which}_avg_us"], 2),
                "timed_launches": r[f"{which}_launches"], "timing": f"HIP events on every {args.timing}th iteration",
                "share_of_solve": round(r[f"{which}_avg_us"] * np.mean(r["iterations"]) /
                                        (1e3 * r["ms_per_solve"]), 3)}
    c4_sys = c5_sys = None
    if pool is not None:
        t_wait = time.time()
        c4_sys = fut_c4.result() if fut_c4 is not None else None
        c5_sys = [f.result() for f in fut_c5]
        pool.shutdown()
        log(f"  background inputs ready (waited {time.time() - t_wait:.1f} s)")
    elif want_c4 or want_c5:
        # --gen-workers 0 (for instance under a profiler): built here
        c4_sys = build_c4() if want_c4 else None
        c5_sys = [build_c5(r) for r in gen.c5_requests()[:args.serve]] if want_c5 else None
    cpu = None
    if not args.no_cpu_baseline:
        model, avail, threads = host_cpu()
        oo = dict(mode=2, tau=1e-3, flags=2, delta=0.0, spd=True, policy=2, shift0=1e-2, border=True)
        log(f"cpu baseline (oracle) on {threads} threads ...")
        cpu = cpu_baseline(system, fp64_its, args.cpu_seconds, oo, threads)
        log(f"  oracle ({threads} threads): {cpu['value']:.5f} solves/s")
        one = cpu_baseline(system, fp64_its, args.cpu_seconds, oo, 1) if threads > 1 else dict(cpu)
        log(f"  oracle (1 thread): {one['value']:.5f} solves/s")
        cpu.update(cpu_model=model, cores_available=avail, single_thread=one["value"],
                   single_thread_sample=one["sample"])
    ceiling = copy_ceiling(torch)
    log(f"  bandwidth ceilings: {ceiling}")
    c4k = run_c4_kernels(sd, torch, c4_sys, args.c4_kernels) if c4_sys is not None else None
    del c4_sys
    serving = (run_serving(sd, torch, gen, c5_sys, args.serve_active, args.serve_modes.split(","), solve_log)
               if c5_sys else None)
    ipm_seq = (run_ipm_sequence(sd, torch, gen, args.c4, args.c4_rows, args.c4_policy, args.c4_precision)
               if args.c4 > 0 else None)
    bbd = run_bbd(sd, torch, gen, args.c3) if args.c3 > 0 else None
    small = run_c1(sd, torch, gen, args.c1) if args.c1 > 0 else None
    line = {
        "metric": METRIC, "value": round(r["solves_per_s"], 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms_per_solve"], 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if best == "fp64" else "f32-inner/f64-refined", "data": "synthetic",
        "config": {"workload": f"{system.name}: M = A D A^T + 1e-8 I, A 200000x500000 (scale {args.scale}), "
                               "8 N(0,1)/col localized + 20 dense cols kept as a low-rank term, D log-uniform "
                               "[1e-6,1e6], 64 blocks, GEOMEAN tau=1e-3 + DROPSUM, ILU(0) with the SHIFT breakdown "
                               "policy, dense columns eliminated as a border (border=1), PCG, tol 1e-8 on the true "
                               "residual; a step = one complete solve from x0 = 0",
                   "n": system.n, "nnz": system.nnz, "nblocks": system.nblocks, "mode": best},
        "p50_ms": round(r["p50_ms"], 2), "p99_ms": round(r["p99_ms"], 2),
        "hbm_gbps": round(r["solve_gbps"], 1), "hbm_gbps_kind": "algorithmic bytes of the whole solve / solve time",
        "iterations": r["iterations"][-1],
        "relres": r["relres"], "roofline": roof, "cpu_baseline": cpu, "bandwidth_ceiling": ceiling,
        "c4_full_size": c4k, "serving": serving, "ipm_sequence": ipm_seq, "bbd": bbd, "c1": small,
        "modes": {k: {kk: (float(f"{vv:.5g}") if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in modes.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
