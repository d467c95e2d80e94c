#!/usr/bin/env python3
"""Benchmark of the space-time heat solver on one MI355X.

One step = one complete FP64 extended-Krylov Galerkin solve (start block,
expansions with the inner Kx / Mx solves, block Gram-Schmidt, reduced
eigensolve and time sweep, projected residual, exact-residual confirmation)
of the 3-D heat problem on the unit cube: trilinear mass and seven-point
stiffness on a 255^3 interior grid (Nh = 16581375), Nt = 4096 steps on
(0, 1], rank-4 separable load, relative Sylvester residual 1e-9, all in FP64.
Inputs are resident in device memory before the timed region; every timed
step re-solves from scratch on the same problem object.  The inner solves run
with the relaxed tolerance of sts_opts.inner_relax (inexact Krylov: a block's
inner solves stop at max(1e-13, min(1e-4, 10^-j tol / r)), r the last
projected residual, j = 2 in 3-D and 1 in 2-D); convergence is still
confirmed on the exact residual.  The CPU baseline and the error gate use the
oracle's sine-mode exact solve on the first time steps.

``--workload heat2d`` runs the 2-D problem instead: P1 on a 511 x 511
interior grid (Nh = 261121), Nt = 1024, rank-2 load (Gaussian-bump fields in
space, trigonometric series in time), relative residual 1e-10; its CPU
baseline and error gate are the oracle's Crank-Nicolson stepper.

Prints one JSON line.  ``value`` is space-time degrees of freedom (Nh * Nt)
per second of wall time.  ``roofline`` reports the kernel with the largest
measured time against its bound (8 TB/s HBM, or 78.6 TFLOP/s FP64 matrix
cores for the exact-residual contraction and the coarse-grid sine-transform
GEMMs), from HIP events attached to every launch of extra solves of the same
workload; ``kernels`` lists all timed kernels.  ``cpu_baseline`` times the CPU
oracle on the first time steps of the same problem, single-threaded, as a
per-step rate (one-off set-up such as a factorisation is timed and reported
apart); those columns also gate the result (relative error <= 1e-8).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "space-time dof/s at rel. error 1e-8; % HBM roofline; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
TRAFFIC_FILES = {"heat2d": os.path.join(ROOT, "profiles", "traffic_2d_n511.json"),
                 "heat3d": os.path.join(ROOT, "profiles", "traffic_3d_n255.json")}
CSRC = os.path.join(ROOT, "paper_1912_10082_amd", "csrc")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


PUBLIC_HEADER = os.path.join(ROOT, "include", "sts.h")


def _file_hashes() -> dict:
    """{source file: first 16 hex digits of its SHA-256} for csrc/ and the
    public header (which the sources include)."""
    paths = {fn: os.path.join(CSRC, fn) for fn in sorted(os.listdir(CSRC))}
    paths["include/sts.h"] = PUBLIC_HEADER
    out = {}
    for fn, p in paths.items():
        with open(p, "rb") as fh:
            out[fn] = hashlib.sha256(fh.read()).hexdigest()[:16]
    return out


def _kernel_sources(hip_name) -> list:
    """The source files a kernel's code depends on: the .hip file that defines
    it and every header."""
    files = [fn for fn in os.listdir(CSRC) if fn.endswith(".h")] + ["include/sts.h"]
    for fn in os.listdir(CSRC):
        if fn.endswith(".hip"):
            with open(os.path.join(CSRC, fn)) as fh:
                if f" {hip_name}(" in fh.read():
                    files.append(fn)
    return sorted(files)


# profiler kernel ids of the library -> HIP kernel names in rocprofv3 output
HIP_KERNELS = {
    "mg_coarse": ["dst_gemm_kernel", "mg_coarse_kernel", "fst_row_kernel", "fst_col_kernel",
                  "coarse3_plane_kernel", "coarse3_z_kernel"],
    "gram": ["gemm_tn_kernel", "gemm_tnw_kernel", "gemm_tn32_kernel"],
    "gram_reduce": ["gemm_tn_reduce", "gemm_tnw_reduce", "gemm_tn32_reduce"],
    "residual": ["residual_kernel"],
    "basis_update": ["gemm_nn_sub_kernel", "gemm_nn_sub4_kernel"],
    "mg_up": ["mg_up_kernel", "mg3_post_kernel", "mg3_post1_kernel", "mg3_post2_kernel"],
    "mg_down": ["mg_down_kernel", "mg3_pre_kernel"],
    "mg_restrict": ["mg3_restrict_kernel"],
    "mass_cheb": ["mass_cheb_kernel", "tensor_mass_kernel", "tensor_mass_x_kernel"],
    "pcg_a": ["pcg_a_kernel", "pcg3_a_kernel"],
    "pcg_b": ["pcg_b_kernel", "pcg3_b_kernel"],
    "stencil": ["apply_kernel"],
}


def _traffic(kernel, path):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs of the same workload (FETCH_SIZE + WRITE_SIZE, each scaled by the
    copy-kernel factor), averaged over the HIP kernels behind the profiler id
    by dispatch count, if every source those kernels depend on is unchanged
    since the counters were taken; else None."""
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    taken, now = d.get("source_sha256_16", {}), _file_hashes()
    ks = d.get("kernels", {})
    tot, cnt = 0.0, 0
    for name in HIP_KERNELS.get(kernel, [kernel]):
        if name not in ks:
            continue
        if any(taken.get(fn) != now.get(fn) for fn in _kernel_sources(name)):
            return None
        n = ks[name].get("dispatches", 1)
        tot += ks[name]["hbm_bytes_per_launch"] * n
        cnt += n
    return tot / cnt if cnt else None


def _coarse_order(n):
    """Order of the exactly solved coarsest multigrid level of an n x n grid:
    halve (n -> (n - 1) / 2) while n > 255, and at least once if n > 63."""
    first = True
    while n > 255 or (first and n > 63):
        n = (n - 1) // 2
        first = False
    return n


def calibrate_copy(mib):
    """A plain device-to-device copy of `mib` MiB, 10 times (one dispatch
    each): the reference that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    torch.cuda.set_device(0)
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(10):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "bytes_read_per_dispatch": n * 8,
                      "bytes_written_per_dispatch": n * 8}), flush=True)
    return 0


def _pmc_per_kernel(path, counter, counts=False):
    """Mean value of `counter` per dispatch, by kernel name, from a rocprofv3
    counter_collection.csv (with counts: also the number of dispatches)."""
    import csv
    import re

    acc = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r.get("Counter_Name") != counter:
                continue
            full = re.sub(r"\(anonymous namespace\)::", "", r["Kernel_Name"])
            name = full.split("(")[0].split("<")[0].split("::")[-1].replace("void ", "").strip()
            a = acc.setdefault(name, [0.0, 0])
            a[0] += float(r["Counter_Value"])
            a[1] += 1
    if counts:
        return {k: (v[0] / v[1], v[1]) for k, v in acc.items()}
    return {k: v[0] / v[1] for k, v in acc.items()}


def summarize_pmc(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_mib, out):
    """Write the per-kernel HBM traffic file from two counter runs of the
    benchmark (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) and the same two runs
    of calibrate_copy."""
    fetch_n = _pmc_per_kernel(fetch_csv, "FETCH_SIZE", counts=True)
    fetch = {k: v[0] for k, v in fetch_n.items()}
    write = _pmc_per_kernel(write_csv, "WRITE_SIZE")
    cf = _pmc_per_kernel(copy_fetch_csv, "FETCH_SIZE")
    cw = _pmc_per_kernel(copy_write_csv, "WRITE_SIZE")
    copy_kib = copy_mib * 1024.0
    # the copy kernel is the one dispatch whose counters are near its size
    f_copy = max(cf.values()) / copy_kib
    w_copy = max(cw.values()) / copy_kib
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        fb = 1024.0 * fetch.get(k, 0.0) / f_copy
        wb = 1024.0 * write.get(k, 0.0) / w_copy
        kernels[k] = {"fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                      "hbm_bytes_per_launch": fb + wb,
                      "dispatches": fetch_n.get(k, (0.0, 0))[1]}
    d = {"source_sha256_16": _file_hashes(),
         "copy_calibration": {"copy_mib": copy_mib, "fetch_factor": f_copy,
                              "write_factor": w_copy},
         "kernels": kernels}
    with open(out, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    print(f"wrote {out}: fetch factor {f_copy:.4f}, write factor {w_copy:.4f}, "
          f"{len(kernels)} kernels", flush=True)
    return 0


def cpu_baseline(w, U_gpu_cols, sample_steps):
    """The oracle on the first `sample_steps` intervals, single-threaded:
    Crank-Nicolson in 2-D (SuperLU factorisation of the step matrix once, then
    one solve per step), the sine-mode exact solve in 3-D (transform of the
    load once, then per step the mode recurrence and an inverse 3-D sine
    transform; a sparse factorisation of a 255^3 step matrix does not fit a
    bounded sample).  The one-off set-up is separated from the per-step cost by
    timing one step and sample_steps + 1 steps.  Returns (seconds per step,
    set-up seconds, relative error of the GPU columns, sample columns)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import exact, fem
    import workloads as wl

    Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
    S = sample_steps
    with threadpool_limits(limits=1):
        if w.dim == 3:
            def run(steps):
                t0 = time.perf_counter()
                U = exact.modal_solve_3d(w.n[0], w.mu, Dt[:steps, :steps], Mt[:steps, :steps],
                                         w.F1, w.F2[:steps])
                return time.perf_counter() - t0, U
        else:
            K, M = fem.spatial_operators(w.dim, w.n[0], w.mu)

            def run(steps):
                t0 = time.perf_counter()
                U = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2, steps=steps)
                return time.perf_counter() - t0, U
        t1, _ = run(1)
        tS, U = run(S + 1)
    per_step = max(tS - t1, 1e-9) / S
    setup = max(t1 - per_step, 0.0)
    err = float(np.linalg.norm(U_gpu_cols - U[:, :U_gpu_cols.shape[1]]) /
                np.linalg.norm(U[:, :U_gpu_cols.shape[1]]))
    return per_step, setup, err, tS


def bench_batch(args) -> int:
    """256 independent 2-D problems of uneven size (grid side 63 / 127 / 255,
    Nt 128..1024, rank 1..3, mu log-uniform in [0.1, 10]) solved to a relative
    residual of 1e-9 through the batch executor, with the worker count picked
    and the inner-solve relaxation picked by the autotuner; the same batch
    with one worker is the sequential reference.  One step = one pass over
    the whole batch."""
    import numpy as np
    import torch

    import paper_1912_10082_amd as sts
    import workloads as wl
    from oracle import exact, fem
    from paper_1912_10082_amd import autotune

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    batch = wl.batch_2d_uneven(count=args.batch_count)
    probs = []
    for w in batch:
        dd, ds, md, ms = sts.time_matrices(wl.time_grid(w.nt, w.T))
        probs.append(sts.Problem(2, w.n[0], w.mu, (dd, ds), (md, ms),
                                 torch.from_numpy(np.asarray(w.F1)).cuda(),
                                 torch.from_numpy(np.asarray(w.F2)).cuda()))
    torch.cuda.synchronize()
    # worker count and inner-solve relaxation (sts_opts.inner_relax) from
    # timed probe runs over a 32-problem subset
    opts = dict(tol=1e-9, max_outer=80, restart=1)
    t0 = time.perf_counter()
    (best, relax), timings = autotune.tune(probs, probe=32, **opts)
    opts["inner_relax"] = relax
    _log(f"autotune {time.perf_counter() - t0:.1f}s: {timings} -> {best} workers, j = {relax}")
    dof = sum(w.nh * w.nt for w in batch)
    res = {}
    for workers in (best, 1):
        with sts.Pool(workers) as pool:
            for i in range(args.warmup):
                pool.solve(probs, **opts)
            lat = []
            for i in range(args.steps):
                t0 = time.perf_counter()
                infos = pool.solve(probs, **opts)
                lat.append(time.perf_counter() - t0)
            _log(f"{workers} workers: {[round(x, 3) for x in lat]} s per batch")
        res[workers] = (sum(lat) / len(lat), infos)
        if workers == best == 1:
            break
    t_best, infos = res[best]
    ok = all(d["status"] == "STS_OK" for d in infos)
    # oracle check on the smaller problems (Crank-Nicolson, CPU)
    errs = []
    for w, pr in zip(batch, probs):
        if w.n[0] == 63 and w.nt <= 256 and len(errs) < 8:
            V, Y = pr.factors()
            K, M = fem.spatial_operators(2, w.n[0], w.mu)
            Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
            U = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
            errs.append(float(np.linalg.norm(V @ Y - U) / np.linalg.norm(U)))
    gate = ok and bool(errs) and max(errs) <= 1e-8
    t_one = res[1][0]
    out = {
        "metric": "batched space-time dof/s (256 independent uneven 2-D problems)",
        "value": dof / t_best, "unit": "dof/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_best, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch2d_uneven_{len(batch)}", "count": len(batch),
                   "sides": [63, 127, 255], "nt": [128, 256, 512, 1024], "p": [1, 2, 3],
                   "tol": opts["tol"], "workers": best, "inner_relax": relax},
        "solves_per_s": len(batch) / t_best,
        "one_worker": {"ms_per_step": 1e3 * t_one, "value": dof / t_one},
        "speedup_vs_one_worker": t_one / t_best,
        "autotune_probe_seconds": {f"w{w}_j{j}": t for (w, j), t in timings.items()},
        "gate_passed": gate, "max_rel_error_sampled": max(errs) if errs else None,
        "errors_sampled": len(errs),
        "outer_its_total": sum(d["outer_its"] for d in infos),
    }
    print(json.dumps(out), flush=True)
    for pr in probs:
        pr.close()
    return 0


def bench_serve(args) -> int:
    """Poisson arrivals (rate --serve-rate, seed 5) over --serve-seconds of
    requests drawn by workloads.serving_mix (50% 1-D with 1000 to 65536 nodes
    log-uniform, 40% 2-D with sides 63 to 511, 10% 3-D with sides 63 to 127;
    Nt log-uniform in [128, 2048]; P in 1..4; mu log-uniform in [0.1, 10]),
    served by --serve-workers workers under a 200 GiB footprint budget, each
    to a relative residual of 1e-8.
    Reports completed solves/s, p50/p99 latency (submission to factors ready)
    and queueing delay; re-solves every 20th request alone to check that its
    factors are bitwise those it got in the mix, and checks the sampled
    requests of modest size against the oracle's Crank-Nicolson solution."""
    import threading

    import numpy as np
    import torch

    import paper_1912_10082_amd as sts
    import workloads as wl
    from oracle import exact, fem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    rng = np.random.default_rng(5)
    gaps = rng.exponential(1.0 / args.serve_rate, size=int(args.serve_rate * args.serve_seconds * 2) + 10)
    arrivals = np.cumsum(gaps)
    arrivals = arrivals[arrivals < args.serve_seconds]
    shapes = wl.serving_mix(len(arrivals), seed=5)
    _log(f"serve: {len(arrivals)} requests over {args.serve_seconds:.0f} s; generating inputs")
    reqs = []
    for sh in shapes:
        w = wl.make_request_workload(*sh)
        dd, ds, md, ms = sts.time_matrices(wl.time_grid(w.nt, w.T))
        reqs.append((w, (dd, ds), (md, ms)))
    # residual 1e-8, the error gate: the exact residual of a 1-D request with
    # tens of thousands of nodes has an FP64 rounding floor near 1e-8
    # (accepted within that floor, sts_solve); each basis grows with its space,
    # so the cap costs no footprint (the slowest 1-D requests, with ~57k
    # nodes and P = 4, take ~150 blocks)
    opts = dict(tol=1e-8, max_outer=250)

    def req_opts(w):
        # relaxed inner solves (sts_opts.inner_relax): j = 2 in 3-D, 1 otherwise;
        # with --serve-mixed, FP32 bulk with FP64 refinement where it applies
        # (3-D grids with n > 63)
        o = dict(opts, inner_relax=2 if w.dim == 3 else 1)
        if args.serve_mixed:
            o["mixed"] = args.mixed_mode
        return o

    budget = 200 << 30
    sample = set(range(0, len(reqs), 20))
    results = [None] * len(reqs)
    kept = {}
    with sts.Server(workers=args.serve_workers, mem_budget=budget) as server:
        # warm-up: one request of each dimension (first-use allocations, code loading)
        for d in (1, 2, 3):
            j = next(i for i, sh in enumerate(shapes) if sh[0] == d)
            w, dt, mt = reqs[j]
            t = server.submit(w.dim, w.n[0], w.mu, dt, mt, w.F1, w.F2, **req_opts(w))
            server.wait(t)
            server.release(t)
        tickets = [None] * len(reqs)
        done_submit = threading.Event()

        def submitter():
            t0 = time.perf_counter()
            for i, (w, dt, mt) in enumerate(reqs):
                delay = arrivals[i] - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                tickets[i] = server.submit(w.dim, w.n[0], w.mu, dt, mt, w.F1, w.F2, **req_opts(w))
            done_submit.set()

        t_start = time.perf_counter()
        th = threading.Thread(target=submitter)
        th.start()
        last_log = t_start
        # collect in completion order (a finished request's memory is
        # released at once, whatever is still running before it)
        pending, nxt, ndone = [], 0, 0
        while ndone < len(reqs):
            while nxt < len(reqs) and tickets[nxt] is not None:
                pending.append(nxt)
                nxt += 1
            still = []
            for i in pending:
                try:
                    res, prob = server.wait(tickets[i], timeout=0.0)
                except sts.STSError:
                    still.append(i)
                    continue
                results[i] = res
                if i in sample and prob is not None:
                    kept[i] = prob.factors()
                server.release(tickets[i])
                ndone += 1
            pending = still
            time.sleep(0.001)
            if time.perf_counter() - last_log > 10:
                last_log = time.perf_counter()
                _log(f"serve: {ndone}/{len(reqs)} done, {server.stats()}")
        th.join()
        t_end = time.perf_counter()
        stats = server.stats()
    wall = t_end - t_start
    ok = [r["status"] == "STS_OK" for r in results]
    lat = sorted(r["latency_seconds"] for r in results)
    qd = sorted(r["queued_seconds"] for r in results)
    pct = lambda a, q: a[min(len(a) - 1, int(q * len(a)))]
    # alone-vs-mixed and oracle checks on the sample
    equal, errs = 0, []
    for i, (V, Y) in kept.items():
        w, dt, mt = reqs[i]
        with sts.Problem(w.dim, w.n[0], w.mu, dt, mt, w.F1, w.F2) as pr:
            pr.solve(**req_opts(w))
            Va, Ya = pr.factors()
        equal += int(np.array_equal(V, Va) and np.array_equal(Y, Ya))
        if w.dim == 3 and w.nh * w.nt <= 1.5e8:
            # 3-D: the oracle's sine-mode exact solve (a sparse factorisation of
            # a 63^3 step matrix does not fit the check's time)
            Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
            U = exact.modal_solve_3d(w.n[0], w.mu, Dt, Mt, w.F1, w.F2)
            errs.append(float(np.linalg.norm(V @ Y - U) / np.linalg.norm(U)))
        elif w.dim < 3 and w.nh * w.nt <= 4e6:
            K, M = fem.spatial_operators(w.dim, w.n[0], w.mu)
            Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
            U = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
            errs.append(float(np.linalg.norm(V @ Y - U) / np.linalg.norm(U)))
    by_dim, svc_dim = {}, {}
    for (w, _, _), r in zip(reqs, results):
        by_dim.setdefault(w.dim, []).append(r["latency_seconds"])
        # admission to factors ready: the request's own time on the GPU, shared
        # with whatever ran beside it
        svc_dim.setdefault(w.dim, []).append(r["latency_seconds"] - r["queued_seconds"])
    dof = sum(w.nh * w.nt for (w, _, _), k in zip(reqs, ok) if k)
    failed = {}
    for (w, _, _), r in zip(reqs, results):
        if r["status"] != "STS_OK":
            key = f"{w.dim}d:{r['status']}"
            failed.setdefault(key, []).append(f"n{w.n[0]}_nt{w.nt}_p{w.p}_res{r['res_true']:.1e}")
    gate = all(ok) and equal == len(kept) and (not errs or max(errs) <= 1e-8)
    out = {
        "metric": "served solves/s and p50/p99 latency (Poisson arrivals, mixed 1-D/2-D/3-D)",
        "value": sum(ok) / wall, "unit": "solves/s", "n_gpus": 1, "steps": len(reqs),
        "warmup": 3, "ms_per_step": 1e3 * wall / max(len(reqs), 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "serve_mix_50_40_10", "rate_per_s": args.serve_rate,
                   "window_s": args.serve_seconds, "workers": args.serve_workers,
                   "mem_budget_bytes": budget, "tol": opts["tol"],
                   "mixed": bool(args.serve_mixed)},
        "latency_ms": {"p50": 1e3 * pct(lat, 0.5), "p99": 1e3 * pct(lat, 0.99)},
        "queued_ms": {"p50": 1e3 * pct(qd, 0.5), "p99": 1e3 * pct(qd, 0.99)},
        "latency_p50_ms_by_dim": {str(d): 1e3 * sorted(v)[len(v) // 2] for d, v in by_dim.items()},
        "service_ms_by_dim": {str(d): {"mean": 1e3 * sum(v) / len(v), "p50": 1e3 * sorted(v)[len(v) // 2],
                                       "sum_s": sum(v), "count": len(v)}
                              for d, v in svc_dim.items()},
        "requests": len(reqs), "completed_ok": sum(ok), "wall_s": wall,
        "space_time_dof_per_s": dof / wall,
        "mem_peak_bytes": stats["mem_peak"],
        "alone_vs_mixed_bitwise_equal": f"{equal}/{len(kept)}",
        "failed": {k: v[:6] for k, v in failed.items()},
        "failed_count": {k: len(v) for k, v in failed.items()},
        "oracle_checked": len(errs), "max_rel_error_sampled": max(errs) if errs else None,
        "gate_passed": gate,
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed solves (heat2d: 50, heat3d: 3)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed solves (heat2d: 2, heat3d: 1)")
    ap.add_argument("--n", type=int, default=None,
                    help="interior nodes per direction (heat2d: 511, heat3d: 255)")
    ap.add_argument("--nt", type=int, default=None, help="time steps (heat2d: 1024, heat3d: 4096)")
    ap.add_argument("--tol", type=float, default=None,
                    help="relative Sylvester residual (heat2d: 1e-10, heat3d: 1e-9)")
    ap.add_argument("--sample-steps", type=int, default=None,
                    help="time steps of the CPU baseline / error gate (heat2d: 48, heat3d: 12)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the profiled solves (no roofline / kernels table)")
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="extra solves with per-dispatch events for the kernel table")
    ap.add_argument("--workload", choices=("heat2d", "heat3d", "batch2d", "serve"),
                    default="heat3d",
                    help="heat3d: the 255^3 x 4096 rank-4 solve in FP64 (default); heat2d: the "
                         "511^2 x 1024 rank-2 solve; batch2d: 256 uneven 2-D problems through the "
                         "batch executor; serve: Poisson arrivals of mixed 1-D / 2-D / 3-D "
                         "requests through the request server")
    ap.add_argument("--mixed", action="store_true",
                    help="heat3d: FP32 bulk with FP64 refinement (sts_opts.mixed): FP32 multigrid "
                         "PCG inside FP64 defect correction for the Kx solves and an FP32 first "
                         "Gram-Schmidt pass; reduced solve and exact residual FP64")
    ap.add_argument("--mixed-mode", type=int, default=2, choices=(1, 2, 3),
                    help="sts_opts.mixed of the mixed-precision runs: 1 = FP32 Kx solves and the FP32 "
                         "first Gram-Schmidt pass, 2 = FP32 Kx solves with the lagged FP64 "
                         "Gram-Schmidt (two reads of V per block), 3 = the FP32 pass only")
    ap.add_argument("--mixed-steps", type=int, default=3,
                    help="heat3d (FP64 run): timed solves of the same problem with sts_opts.mixed, "
                         "reported as mixed_precision with their error against the FP64 run "
                         "(0 = skip)")
    ap.add_argument("--precond-fp32", action="store_true",
                    help="heat3d: multigrid V-cycle vectors in FP32 inside FP64 CG "
                         "(sts_opts.precond_fp32); the default run is FP64 throughout")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=20.0, help="requests per second")
    ap.add_argument("--serve-seconds", type=float, default=30.0, help="arrival window")
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-mixed", action="store_true",
                    help="serve: FP32 bulk with FP64 refinement (sts_opts.mixed) for the requests "
                         "it applies to")
    ap.add_argument("--calibrate-copy", type=int, metavar="MIB", default=0,
                    help="only run a plain MIB-MiB device copy (counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=5,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV", "MIB"),
                    help="only write the HBM traffic file from rocprofv3 counter runs")
    args = ap.parse_args()
    d3 = args.workload == "heat3d"
    if args.n is None:
        args.n = 255 if d3 else 511
    if args.nt is None:
        args.nt = 4096 if d3 else 1024
    if args.tol is None:
        args.tol = 1e-9 if d3 else 1e-10
    if args.steps is None:
        args.steps = 3 if d3 else 50
    if args.warmup is None:
        args.warmup = 1 if d3 else 2
    if d3 and args.profile_steps == 3:
        args.profile_steps = 1
    if args.sample_steps is None:
        args.sample_steps = 12 if d3 else 48
    if args.summarize_pmc:
        f, wr, cf, cw, mib = args.summarize_pmc
        return summarize_pmc(f, wr, cf, cw, int(mib), TRAFFIC_FILES[args.workload])
    if args.calibrate_copy:
        return calibrate_copy(args.calibrate_copy)
    if args.gpus == 1 and args.workload == "batch2d":
        return bench_batch(args)
    if args.gpus == 1 and args.workload == "serve":
        return bench_serve(args)
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "the solver has no multi-GPU path", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1912_10082_amd as sts
    import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    p_rank = 4 if d3 else 2
    if d3:
        w = wl.heat_3d_separable(n=args.n, nt=args.nt, p=p_rank, seed=3)
    else:
        w = wl.heat_2d_bumps(n=args.n, nt=args.nt, p=p_rank, seed=2)
    t = wl.time_grid(w.nt, w.T)
    dd, ds, md, ms = sts.time_matrices(t)
    F1 = torch.from_numpy(np.asarray(w.F1)).cuda()
    F2 = torch.from_numpy(np.asarray(w.F2)).cuda()
    torch.cuda.synchronize()
    prob = sts.Problem(w.dim, w.n[0], w.mu, (dd, ds), (md, ms), F1, F2)
    # inner solves relaxed as the residual falls (inexact Krylov): each block's
    # solves stop at max(1e-13, min(1e-4, 10^-j tol / r)); the exact residual
    # still decides convergence.  j = 1 in 2-D, 2 in 3-D (measured best: with
    # j = 1 the 3-D solve needs a second exact residual, 0.7 s).  The basis
    # grows with the space (the 255^3 rank-4 run holds about 424 of the 808
    # columns max_outer allows)
    opts = dict(tol=args.tol, restart=1, max_outer=100 if d3 else 150, inner_relax=2 if d3 else 1)
    if args.precond_fp32:
        # mixed precision: the 3-D multigrid V-cycle stores its vectors in FP32
        # inside FP64 CG (sts_opts.precond_fp32); everything else stays FP64
        opts["precond_fp32"] = 1
    if args.mixed:
        opts["mixed"] = args.mixed_mode
    for i in range(args.warmup):
        info = prob.solve(**opts)
        _log(f"warmup {i}: {info['status']} outer={info['outer_its']} k={info['k']} "
             f"{info['seconds']:.3f}s")
    torch.cuda.synchronize()
    lat, infos = [], []
    for i in range(args.steps):
        t0 = time.perf_counter()
        info = prob.solve(**opts)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        infos.append(info)
        if i < 3 or i == args.steps - 1:
            _log(f"step {i}: {info['status']} outer={info['outer_its']} k={info['k']} "
                 f"res_true={info['res_true']:.2e} {lat[-1]:.3f}s")
    # Kernel durations: the same solve again with a start/stop event attached
    # to every dispatch.  The events widen the gaps between launches (so
    # these solves are not timed), not the kernels' own durations.
    ksum = {}
    prof_steps = 0 if args.no_profile else args.profile_steps
    for i in range(prof_steps):
        prob.solve(profile=1, **opts)
        torch.cuda.synchronize()
        for name, (sec, n, by) in prob.kernel_profile().items():
            a = ksum.setdefault(name, [0.0, 0, 0.0])
            a[0] += sec
            a[1] += n
            a[2] += by
    total = sum(lat)
    dof = w.nh * w.nt
    value = dof * args.steps / total
    last = infos[-1]
    roofline = None
    kernels = None
    if ksum:
        # dominant kernel by measured time; its algorithmic bytes (or flops) per
        # launch over its average launch duration
        ktot = sum(v[0] for v in ksum.values())
        name, (sec, n, by) = max(ksum.items(), key=lambda kv: kv[1][0])
        kernels = {k: {"ms_per_solve": 1e3 * v[0] / prof_steps,
                       "launches_per_solve": v[1] / prof_steps, "kernel_time_share": v[0] / ktot,
                       "GB_per_s": (v[2] / v[0] / 1e9) if v[0] > 0 and v[2] > 0 else None}
                   for k, v in sorted(ksum.items(), key=lambda kv: -kv[1][0]) if v[1] > 0}
        avg_us = 1e6 * sec / max(n, 1)
        common = {"avg_launch_us": avg_us, "launches_per_solve": n / prof_steps,
                  "kernel_time_share": sec / ktot,
                  "measured": f"HIP events on every dispatch of {prof_steps} more solves "
                              "of the same workload after the timed steps"}
        flops = None
        if name == "residual":
            # ||[F1, Kx V, Mx V] B^T||: 2 Nh m Nt flops per launch on the FP64 matrix cores
            # (m = P + 2k), or 2 Nh m^2 when B was first reduced to its QR factor
            m = p_rank + 2 * last["k"]
            qr = ksum.get("residual_qr", [0.0, 0, 0.0])[1] > 0
            flops = 2.0 * w.nh * m * (m if qr else w.nt) * n
        elif name == "mg_coarse" and not d3 and (_coarse_order(w.n[0]) + 1) not in (128, 256):
            # exact coarse solve as m x m GEMMs on the matrix cores (operands
            # L2-resident, 2 m^3 flops per 24 m^2 algorithmic bytes per column);
            # orders m = 127, 255 use fast sine transforms instead (memory-bound)
            m = _coarse_order(w.n[0])
            flops = by * m / 12.0
        if flops is not None:
            achieved = flops / sec / 1e12
            roofline = {"kernel": name, "bound": "mfma", "achieved": round(achieved, 2),
                        "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                        "traffic": _traffic(name, TRAFFIC_FILES[args.workload]),
                        "alg_flops_per_launch": flops / max(n, 1), **common}
        else:
            achieved = by / sec / 1e9
            roofline = {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": _traffic(name, TRAFFIC_FILES[args.workload]),
                        "alg_bytes_per_launch": by / max(n, 1), **common}
            if name == "gram" and "gram_reduce" in ksum:
                # the contraction as a whole: the streaming launch plus the
                # launch that sums its per-chunk partial products
                rsec = ksum["gram_reduce"][0]
                roofline["frac_with_reduce"] = round(by / (sec + rsec) / 1e9 / HBM_PEAK_GBS, 4)
    gate = last["status"] == "STS_OK" and last["res_true"] <= args.tol
    S = min(args.sample_steps, w.nt - 1)
    U_gate = None if args.no_cpu_baseline else prob.solution_columns(list(range(S)))
    mixed = None
    if d3 and not args.mixed and args.mixed_steps > 0:
        cols = sorted(set(int(round(x)) for x in np.linspace(0, w.nt - 1, 64)))
        Uf = prob.solution_columns(cols, device=True)
        # the same problem with FP32 bulk work and FP64 refinement
        # (sts_opts.mixed), gated at relative error 1e-8 against this FP64 run
        # on sampled time columns
        mopts = dict(opts, mixed=args.mixed_mode)
        minfo = prob.solve(**mopts)   # first mixed solve: the FP32 copy of V is allocated
        torch.cuda.synchronize()
        mlat = []
        for i in range(args.mixed_steps):
            t0 = time.perf_counter()
            minfo = prob.solve(**mopts)
            torch.cuda.synchronize()
            mlat.append(time.perf_counter() - t0)
        _log(f"mixed: {minfo['status']} outer={minfo['outer_its']} k={minfo['k']} "
             f"res_true={minfo['res_true']:.2e} {[round(x, 3) for x in mlat]} s")
        Um = prob.solution_columns(cols, device=True)
        merr = float(torch.linalg.norm(Um - Uf) / torch.linalg.norm(Uf))
        mt = sum(mlat) / len(mlat)
        mixed = {"dtype": "f32+f64_refine", "sts_opts_mixed": args.mixed_mode,
                 "value": w.nh * w.nt / mt, "unit": "dof/s",
                 "ms_per_step": 1e3 * mt, "steps": len(mlat),
                 "rel_error_vs_fp64_run": merr, "error_columns": len(cols),
                 "res_true": minfo["res_true"], "outer_its": minfo["outer_its"], "k": minfo["k"],
                 "inner_its_K": minfo["inner_its_K"], "inner_its_fp32": minfo["inner_its_fp32"],
                 "defect_rounds": minfo["defect_rounds"],
                 "gate_passed": bool(minfo["status"] == "STS_OK" and minfo["res_true"] <= args.tol
                                     and merr <= 1e-8)}
        del Um, Uf
    cpu = None
    err = None
    if not args.no_cpu_baseline:
        per_step, setup, err, total_s = cpu_baseline(w, U_gate, S)
        gate = gate and err <= 1e-8
        if d3:
            sample = (f"first {S + 1} of {w.nt} time steps of the same {w.n[0]}^3 x {w.nt} problem "
                      f"by the oracle's sine-mode solve, single-threaded (SciPy FFTs, NumPy with "
                      f"BLAS threads limited to 1): {per_step:.2f} s per step, {setup:.2f} s "
                      f"one-off transform of the load; {total_s:.1f} s in all")
        else:
            sample = (f"first {S + 1} of {w.nt} Crank-Nicolson steps of the same {w.n[0]}^2 x "
                      f"{w.nt} problem, single-threaded SciPy SuperLU: {setup:.2f} s factorisation "
                      f"once, then {1e3 * per_step:.1f} ms per step; {total_s:.1f} s in all")
        cpu = {"value": w.nh / per_step, "unit": "dof/s", "cores": 1, "kind": "oracle",
               "sample": sample, "seconds_per_step": per_step, "setup_seconds": setup,
               "host_cores_available": len(os.sched_getaffinity(0))}
    lat_ms = sorted(1e3 * x for x in lat)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "dof/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32+f64_refine" if args.mixed else
                  "f64+f32_precond" if args.precond_fp32 else "f64"),
        "data": "synthetic",
        "config": ({"workload": f"heat3d_q1_7pt_{w.n[0]}^3_nt{w.nt}_rank4_tol{args.tol:g}"
                                + ("_mixed" if args.mixed else "_mg_fp32" if args.precond_fp32 else ""),
                    "nh": w.nh, "nt": w.nt, "p": 4, "tol": args.tol, "seed": 3} if d3 else
                   {"workload": f"heat2d_p1_courant_{w.n[0]}x{w.n[0]}_nt{w.nt}_rank2_tol{args.tol:g}",
                    "nh": w.nh, "nt": w.nt, "p": 2, "tol": args.tol, "seed": 2}),
        "latency_ms": {"p50": lat_ms[len(lat_ms) // 2],
                       "p99": lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))]},
        "gate_passed": bool(gate),
        "rel_error_vs_oracle_sample": err,
        "res_true": last["res_true"],
        "outer_its": last["outer_its"],
        "k": last["k"],
        "inner_its_K": last["inner_its_K"],
        "inner_its_M": last["inner_its_M"],
        "inner_its_fp32": last["inner_its_fp32"],
        "defect_rounds": last["defect_rounds"],
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "mixed_precision": mixed,
    }
    print(json.dumps(out), flush=True)
    prob.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
