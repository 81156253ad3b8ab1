"""Benchmark: solves/s of the accelerated Jacobi-type solver on one MI355X.

Default workload: the 3D 7-point Dirichlet Laplacian on a 128^3 grid
(n = 2,097,152, nnz = 14,581,760), float64, b = Q x* with x* ~ N(0,1)
(seed 1002), x^0 = 0, restart on, K_0 = 2, solved to a confirmed relative
residual <= 1e-8.  One step = one complete solve (all iterations of the
fused-pass launches), inputs resident in HBM, system set up beforehand.

Prints one JSON line with the solve throughput, p50/p99 latency, the
roofline figures of the fused iteration kernel k_pass64 (algorithmic bytes
per launch / its mean launch duration from HIP events on the solve's stream),
the HBM traffic per launch from the committed counter runs (null when the
kernel sources changed since), and the CPU oracle baseline.

    python bench.py [--steps K] [--warmup W] [--workload laplace3d_128|poisson2d_64|laplace3d_160|laplace3d_192]
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

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
CSRC = os.path.join(ROOT, "paper_2407_03272_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


# The files that define the fused pass kernel k_pass64 (its code, the layout it reads and its partition of
# slices over workgroups).  Host-side files only choose its instance and grid, which the traffic record
# names itself.
PASS_KERNEL_SOURCES = ("naj_device.h", "naj_solve.h", "naj_partition.h")


def strip_comments(text: str) -> str:
    """C++ source without its comments and trailing blanks (the pass kernel's sources hold no string
    literal with a comment marker), so a comment edit leaves the key of the counter records unchanged."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_source_hash(read=None) -> str:
    """SHA-256 of the pass kernel's sources without comments; `read(name)` supplies a source's text
    (default: the file in the package)."""
    import hashlib
    h = hashlib.sha256()
    for name in PASS_KERNEL_SOURCES:
        text = read(name) if read else open(os.path.join(CSRC, name), encoding="utf-8").read()
        h.update(name.encode())
        h.update(strip_comments(text).encode())
    return h.hexdigest()


def measured_traffic(workload: str, grid: int | None = None, value_bytes: int | None = None):
    """HBM bytes per pass from the committed rocprofv3 counter runs, or None when none exist for this
    workload, the pass kernel's sources changed since they were taken, or the pass ran on another grid or
    read values of another size."""
    path = os.path.join(PROFILES, f"k_pass64_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if grid is not None and rec.get("grid") not in (None, grid):
        return None
    if value_bytes is not None and rec.get("value_bytes", 8) != value_bytes:
        return None
    return rec["traffic_bytes_per_pass"]


def bytes_per_iteration(n: int, nnz: int, s_v: int = 8, s_x: int = 8, k: int = 1, jb: int = 0,
                        nnz_off: int = 0) -> int:
    """Algorithmic bytes of one fused pass, CSR int32 yardstick: values + int32 columns, int32 row pointers,
    and four vector streams (read x^{t-1}, read y^t / x^{t-2}, read b, write x^t); with a block J of jb-row
    blocks, each row also reads its row of the block's inverse (jb values).  With nnz_off > 0: the bytes the
    layout itself moves, without the column indices of the nnz_off nonzeros held in column-offset slices
    (their columns follow from the slice's offset list)."""
    return s_v * nnz + 4 * (nnz - nnz_off) + 4 * (n + 1) + 4 * k * s_x * n + jb * s_x * n


def bytes_per_residual(n: int, nnz: int, nnz_off: int = 0, s_v: int = 8) -> int:
    """Algorithmic bytes of one float64 residual pass r = b - Q x: matrix, row pointers, read x and b
    (s_v bytes per value: 4 where the layout reads the exact float32 copy)."""
    return s_v * nnz + 4 * (nnz - nnz_off) + 4 * (n + 1) + 2 * 8 * n


def bytes_per_refinement_residual(n: int, nnz: int, nnz_off: int = 0, s_v: int = 8) -> int:
    """Float64 residual pass of the mixed loop with the update fused: matrix, row pointers, read x (f64), d (f32)
    and b, write x + d (f64) and fl32(r) (f32)."""
    return s_v * nnz + 4 * (nnz - nnz_off) + 4 * (n + 1) + 8 * n + 4 * n + 8 * n + 8 * n + 4 * n


def solve_bytes(n: int, nnz: int, info, mixed: bool, jb: int = 0, nnz_off: int = 0, vb: int = 8) -> int:
    """Bytes of a whole solve from its pass counts (norm of b = 8n bytes), with vb bytes per matrix value
    read by the float64 passes (the element size s_v of the yardstick): the CSR yardstick, or with nnz_off
    the bytes the layout moves."""
    if not mixed:
        it = info.iterations
        conf = info.passes - it - 1
        return (8 * n + it * bytes_per_iteration(n, nnz, s_v=vb, jb=jb, nnz_off=nnz_off)
                + conf * bytes_per_residual(n, nnz, nnz_off, s_v=vb))
    return (8 * n + info.iterations * bytes_per_iteration(n, nnz, s_v=4, s_x=4, jb=jb, nnz_off=nnz_off)
            + info.confirmations * bytes_per_refinement_residual(n, nnz, nnz_off, s_v=vb))


def make_workload(name: str):
    from paper_2407_03272_amd import workloads as W
    if name == "laplace3d_128":
        return W.poisson3d_128()
    if name == "laplace3d_160":
        return W.poisson_system((160, 160, 160), 1006, name="laplace3d_160")
    if name == "laplace3d_192":
        return W.poisson_system((192, 192, 192), 1007, name="laplace3d_192")
    if name == "poisson2d_64":
        return W.poisson2d_64()
    if name == "chunglu_4m":
        return W.chung_lu_laplacian()
    if name.startswith("sdd_"):       # the Section 4.1 system (n+1) I - 1 1^T, b = 1 (dense rows)
        return W.sdd_system(int(name[4:]))
    raise SystemExit(f"unknown workload {name}")


def host_cpu() -> dict:
    """Host CPU facts for the baseline: logical CPUs this process may use, and the model name."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"nproc": nproc, "cpu_model": model, "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(sysobj, iterations_needed: int, sample_iters: int, jblock=None, stop_kw=None,
                 progress=None) -> dict:
    """The CPU oracle (as it is) on the same solve.

    Diagonal J with the residual stop: the multi-core C oracle (OpenMP over rows) runs the whole
    float64 solve on every thread OpenMP gives it (OMP_NUM_THREADS), timed around the solve with
    setup excluded, repeated while the repeats take under about 8 s (median reported); a one-thread
    run over the first `sample_iters` iterations is scaled to one solve beside it.  Block J or the
    objective stop: the numpy/scipy oracle on one thread over the first `sample_iters` iterations,
    scaled to one solve."""
    info = host_cpu()
    if jblock or stop_kw:
        from threadpoolctl import threadpool_limits

        import oracle as O
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            r = O.accelerated_jacobi(sysobj.rowptr, sysobj.colidx, sysobj.vals, sysobj.b, tol=1e-8,
                                     max_iter=sample_iters, jblock=jblock, **(stop_kw or {}))
            dt = time.perf_counter() - t0
        per_iter = dt / max(1, len(r.hist))
        return {"value": 1.0 / (per_iter * iterations_needed), "unit": "solves/s", "cores": 1, "kind": "oracle",
                "sample": f"first {len(r.hist)} of {iterations_needed} iterations of the same float64 solve "
                          f"({dt:.1f} s, {per_iter * 1e3:.1f} ms/iteration, numpy/scipy single thread), "
                          f"scaled to one full solve", **info}
    from oracle import cpu_omp
    times, r = [], None
    t_all = time.perf_counter()
    while len(times) < 5 and (len(times) < 1 or time.perf_counter() - t_all < 8.0):
        r = cpu_omp.solve(sysobj.rowptr, sysobj.colidx, sysobj.vals, sysobj.b, tol=1e-8, max_iter=20000,
                          threads=0, hist_cap=0)
        times.append(r.seconds)
        if progress:
            progress(f"cpu oracle ({r.threads} threads): {r.seconds:.2f} s, {r.iterations} iterations")
    med = float(np.median(times))
    one = cpu_omp.solve(sysobj.rowptr, sysobj.colidx, sysobj.vals, sysobj.b, tol=1e-8,
                        max_iter=min(sample_iters, max(1, r.iterations)), threads=1, hist_cap=0)
    per_iter1 = one.seconds / max(1, one.iterations)
    return {"value": 1.0 / med, "unit": "solves/s", "cores": r.threads, "kind": "oracle",
            "sample": f"{len(times)} complete float64 solves of the same system by the C oracle "
                      f"(OpenMP over rows, {r.threads} threads; {r.iterations} iterations, relres {r.relres:.3g}, "
                      f"status {r.status}), median {med:.2f} s",
            "iterations": r.iterations, "seconds_median": med,
            "single_thread": {"value": 1.0 / (per_iter1 * r.iterations), "unit": "solves/s", "cores": 1,
                              "sample": f"first {one.iterations} iterations on one thread "
                                        f"({one.seconds:.2f} s, {per_iter1 * 1e3:.2f} ms/iteration), "
                                        f"scaled to {r.iterations} iterations"},
            **info}


def attainable_bandwidth(progress=None) -> dict:
    """The GPU's attainable streaming rates, measured by the library's probe kernel (naj_bandwidth_probe:
    16 KB blocks taken by the workgroups in turn, 16-byte accesses, over 1 GiB, mean of 20 launches timed
    with HIP events on the launching stream): read only, copy (read + write bytes) and write only, beside
    the 8 TB/s published peak."""
    import torch
    from paper_2407_03272_amd import naj
    out = {}
    for mode in (0, 1, 2):
        r = naj.bandwidth_probe(mode, 1 << 30, 20)
        out[r["mode"] + "_gbps"] = r["gbps"]
        if mode == 1:
            assert r["copy_exact"], "bandwidth probe copy mismatch"
    torch.cuda.empty_cache()
    out["best_gbps"] = max(out["read_gbps"], out["copy_gbps"], out["write_gbps"])
    out["best_frac_of_peak"] = out["best_gbps"] / HBM_PEAK_GBS
    out["kernel"] = ("naj_bandwidth_probe (k_bw_probe), 1 GiB in 16 KB blocks taken by the workgroups in turn, "
                     "16-byte accesses (non-temporal loads; copy: non-temporal stores), mean of 20 launches")
    if progress:
        progress(f"attainable bandwidth: read {out['read_gbps']:.0f}, copy {out['copy_gbps']:.0f}, "
                 f"write {out['write_gbps']:.0f} GB/s")
    return out


def component_mean_free(rowptr, colidx, vals, x: np.ndarray) -> np.ndarray:
    """x minus its J-weighted mean on each connected component of the matrix graph (J = absolute row
    sums, 1 on zero rows): the part of x outside the null space of a graph Laplacian, where the
    method keeps the J-weighted sum of the starting point on every component."""
    import scipy.sparse as sps
    from scipy.sparse.csgraph import connected_components
    n = len(rowptr) - 1
    A = sps.csr_matrix((np.abs(vals), colidx, rowptr), shape=(n, n))
    J = np.asarray(A.sum(axis=1)).ravel()
    J[J == 0] = 1.0
    nc, lab = connected_components(A, directed=False)
    mean = np.bincount(lab, weights=J * x, minlength=nc) / np.bincount(lab, weights=J, minlength=nc)
    return x - mean[lab]


def bench_fe_batch(args, progress):
    """512 P1 finite-element systems (2D/3D, n log-uniform in [1e3, 2e5], lognormal coefficients), 8 right-hand
    sides each, solved together in mixed precision by graph-replayed batch passes with autotuned tiles.
    One step = the whole batch (4096 solves).  Compared with the same batch in float64 and with plain float64
    one-system-at-a-time solves (a sample of them, scaled)."""
    import torch
    from paper_2407_03272_amd import naj
    from paper_2407_03272_amd import workloads as W

    nrhs = 8
    systems = W.fe_batch(args.nsys, nrhs=nrhs, workers=min(8, os.cpu_count() or 1))
    progress(f"generated {len(systems)} systems, sum n = {sum(x.n for x in systems)}, "
             f"sum nnz = {sum(x.nnz for x in systems)}")
    syss = [naj.System(x.rowptr, x.colidx, x.vals) for x in systems]
    progress("systems created")
    reps = {}
    for x, sm in zip(systems, syss):
        key = (sm.info()["layout"], int(np.log2(x.n)), int(round(x.nnz / x.n)))
        reps.setdefault(key, sm)
    prec = naj.NAJ_MIXED if args.precision == "mixed" else naj.NAJ_FP64
    tiles = {}
    for key, sm in sorted(reps.items()):
        tiles[str(key)] = naj.autotune_tiles(sm, nrhs, passes=20, precision=prec)
    progress(f"autotuned {len(reps)} feature keys")
    bs = [torch.as_tensor(x.b).cuda() for x in systems]

    def run_batch(precision, steps, warmup):
        bt = naj.Batch(syss, [nrhs] * len(syss), tol=1e-8, max_iter=20000, precision=precision)
        outs = [torch.empty_like(b) for b in bs]
        for _ in range(warmup):
            t0 = time.perf_counter()
            _, winf, _ = bt.solve(bs, outs=outs)
            progress(f"warm-up batch solve ({'mixed' if precision == naj.NAJ_MIXED else 'fp64'}): "
                     f"{time.perf_counter() - t0:.2f} s, max iterations {max(i.iterations for i in winf)}")
        torch.cuda.synchronize()
        times, kms = [], []
        t_all = time.perf_counter()
        for _ in range(steps):
            t0 = time.perf_counter()
            _, infos, ms = bt.solve(bs, outs=outs)
            times.append(time.perf_counter() - t0)
            kms.append(ms)
            progress(f"batch solve: {times[-1]:.2f} s")
            bad = [i.status for i in infos if i.status != 0]
            if bad:
                raise SystemExit(f"batch: {len(bad)} instances did not converge")
        torch.cuda.synchronize()
        total = time.perf_counter() - t_all
        info = bt.info()
        bt.close()
        return total, times, kms, infos, info, outs

    total, times, kms, infos, binfo, xs_main = run_batch(prec, args.steps, args.warmup)
    ninst = len(infos)
    progress(f"batch: {total / args.steps * 1e3:.1f} ms per {ninst} solves")
    # algorithmic bytes: matrix once per system pass, vectors per instance pass
    alg = 0
    for i, x in enumerate(systems):
        inf = infos[i * nrhs:(i + 1) * nrhs]
        n, nnz = x.n, x.nnz
        if prec == naj.NAJ_MIXED:
            alg += max(v.iterations for v in inf) * (8 * nnz + 4 * (n + 1))
            alg += max(v.confirmations for v in inf) * (12 * nnz + 4 * (n + 1))
            alg += sum(v.iterations * 16 * n + v.confirmations * 32 * n + 8 * n for v in inf)
        else:
            alg += max(v.passes for v in inf) * (12 * nnz + 4 * (n + 1))
            alg += sum(v.passes * 32 * n for v in inf)
    kernel_s = float(np.mean(kms)) / 1e3
    achieved = alg / kernel_s / 1e9
    line = {
        "metric": "solves/s + HBM GB/s at relres 1e-8 vs plain FP64; p50/p99 solve latency",
        "value": ninst * args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == naj.NAJ_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": f"{len(systems)} P1 finite-element systems (2D/3D, n log-uniform 1e3..2e5, seed 1004) x "
                               f"{nrhs} right-hand sides, one batch of graph-replayed passes, autotuned tiles, "
                               f"{'float32 inner + float64 refinement' if prec == naj.NAJ_MIXED else 'float64'}, "
                               f"relres <= 1e-8 per solve; one step = all {ninst} solves",
                   "systems": len(systems), "nrhs": nrhs, "sum_n": int(sum(x.n for x in systems)),
                   "sum_nnz": int(sum(x.nnz for x in systems)), "tiles": binfo["ntiles"], "grid": binfo["grid"],
                   "tile_table": tiles,
                   "iterations_min_median_max": [int(np.min([i.iterations for i in infos])),
                                                 int(np.median([i.iterations for i in infos])),
                                                 int(np.max([i.iterations for i in infos]))]},
        "p50_ms": float(np.percentile(times, 50) * 1e3),
        "p99_ms": float(np.percentile(times, 99) * 1e3),
        "kernel_ms": float(np.mean(kms)),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_batch_pass (one launch per batch pass, graph-replayed)",
                     "algorithmic_bytes_per_batch_solve": alg},
    }
    if not args.no_compare:
        other = naj.NAJ_FP64 if prec == naj.NAJ_MIXED else naj.NAJ_MIXED
        ctot, ctimes, ckms, cinfos, _, xs_other = run_batch(other, max(2, args.steps // 2), 1)
        # every instance's mixed answer against its float64 answer (both to relres 1e-8)
        errs = []
        for a, c in zip(xs_main, xs_other):
            d = torch.linalg.vector_norm((a - c).reshape(a.shape[0], -1), dim=0)
            errs.append((d / torch.linalg.vector_norm(c.reshape(c.shape[0], -1), dim=0)).cpu().numpy())
        errs = np.concatenate(errs)
        line["compare_batch"] = {"precision": "fp64" if other == naj.NAJ_FP64 else "mixed",
                                 "solves_per_s": ninst * len(ctimes) / ctot,
                                 "ms_per_batch": ctot / len(ctimes) * 1e3,
                                 "rel_err_mixed_vs_fp64": {"instances": int(errs.size),
                                                           "median": float(np.median(errs)),
                                                           "max": float(np.max(errs))}}
        progress("batch comparison done")
        # plain float64, one system and one right-hand side at a time (every 16th system, all 8 rhs)
        sample = list(range(0, len(systems), 16))
        t0 = time.perf_counter()
        nsol = 0
        for i in sample:
            for j in range(nrhs):
                bj = bs[i][:, j].contiguous()
                _, inf = syss[i].solve(bj, tol=1e-8, max_iter=20000, hist_cap=0)
                nsol += 1
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # scale the sample to the whole batch by the sampled systems' share of rows
        share = sum(systems[i].n for i in sample) / sum(x.n for x in systems)
        line["compare_one_at_a_time"] = {"precision": "fp64", "sampled_solves": nsol,
                                         "sample_seconds": dt,
                                         "solves_per_s_est": ninst / (dt / share)}
        progress("one-at-a-time comparison done")
    return line


def run_server(naj, reqs, budget, slots, closed_loop, progress, label):
    """Replays the trace through a server: admission as requests arrive (all at t=0 when
    closed_loop), continuous batching, result copied to the host.  Returns per-request
    latencies (arrival -> answer on the host) and the makespan."""
    import torch
    from collections import deque
    srv = naj.Server(budget, slots, max_rhs=1, precision=naj.NAJ_MIXED, tol=1e-8, max_iter=20000)
    arr = np.zeros(len(reqs)) if closed_loop else np.array([r["t"] for r in reqs])
    lat = np.full(len(reqs), np.nan)
    tickets, queue = {}, deque()
    nxt, ndone, busy_max, bad = 0, 0, 0, 0
    last_report = 0.0
    host = {"admit": 0.0, "step": 0.0, "result": 0.0, "steps": 0}
    staged = None
    kept = []   # every 10th answer, checked against its tolerance after the timed loop
    t0 = time.perf_counter()
    while ndone < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arr[nxt] <= now:
            queue.append(nxt)
            nxt += 1
        ta = time.perf_counter()
        while queue:
            i = queue[0]
            r = reqs[i]
            if staged is None or staged[0] != i:   # upload once; a busy server is retried with the same copies
                staged = (i, srv.stage(r["sys"].rowptr, r["sys"].colidx, r["sys"].vals, r["b"]))
            rp, ci, va, bb, _, _ = staged[1]
            t = srv.admit(rp, ci, va, bb, tol=r["tol"])
            if t is None:
                break
            tickets[t] = i
            queue.popleft()
            staged = None
        tb = time.perf_counter()
        busy_max = max(busy_max, len(queue))
        active = len(tickets) > 0
        fin = srv.step(1 if active else 0)
        tc = time.perf_counter()
        for t in fin:
            i = tickets.pop(t)
            x, infos = srv.result(t)
            xh = x.cpu()
            lat[i] = time.perf_counter() - t0 - arr[i]
            bad += int(infos[0].status != 0)
            ndone += 1
            if i % 10 == 0:
                kept.append((i, xh.numpy()))
        td = time.perf_counter()
        host["admit"] += tb - ta
        host["step"] += tc - tb
        host["result"] += td - tc
        host["steps"] += 1
        if not active and not queue and nxt < len(reqs):
            wait = arr[nxt] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.002))
        if time.perf_counter() - t0 - last_report > 5.0:
            last_report = time.perf_counter() - t0
            progress(f"{label}: {ndone}/{len(reqs)} done, {len(tickets)} in flight, {len(queue)} queued")
    makespan = time.perf_counter() - t0
    srv.close()
    progress(f"{label}: host seconds admit {host['admit']:.2f}, step {host['step']:.2f}, result {host['result']:.2f} "
             f"over {host['steps']} loop turns, makespan {makespan:.2f}")
    import scipy.sparse as sps
    for i, xh in kept:   # the answers meet their tolerances by an independent float64 product
        s, b = reqs[i]["sys"], reqs[i]["b"]
        Q = sps.csr_matrix((s.vals, s.colidx, s.rowptr), shape=(s.n, s.n))
        if np.linalg.norm(b - Q @ xh) / np.linalg.norm(b) > reqs[i]["tol"]:
            bad += 1
    progress(f"{label}: {len(kept)} sampled answers checked")
    return lat, makespan, busy_max, bad, dict(kept)


def bench_serve(args, progress):
    """Serving loop under a Poisson request trace (continuous batching, mixed precision)."""
    import torch
    from paper_2407_03272_amd import naj
    nreq, warm = args.serve_requests, min(200, args.serve_requests // 10)
    from paper_2407_03272_amd import workloads as W
    reqs = W.serve_trace(nreq, workers=min(16, os.cpu_count() or 1))
    progress(f"trace: {nreq} requests over {reqs[-1]['t']:.2f} s, "
             f"{sum(r['fe'] for r in reqs)} finite-element, {sum(not r['fe'] for r in reqs)} Laplacians")
    budget = int(args.serve_budget_mb) << 20
    # open loop at the trace's arrival times
    lat, span, qmax, bad, served = run_server(naj, reqs, budget, args.serve_slots, False, progress, "open loop")
    if bad:
        raise SystemExit(f"serve: {bad} requests did not converge or missed their tolerance")
    L = lat[warm:] * 1e3
    first = reqs[warm]["t"]
    achieved = (nreq - warm) / (span - first)
    progress(f"open loop: p50 {np.percentile(L, 50):.1f} ms, p99 {np.percentile(L, 99):.1f} ms, "
             f"{achieved:.1f} solves/s")
    # closed loop: every request queued at t = 0 (saturation throughput)
    clat, cspan, _, cbad, _ = run_server(naj, reqs, budget, args.serve_slots, True, progress, "closed loop")
    if cbad:
        raise SystemExit(f"serve (closed loop): {cbad} requests did not converge or missed their tolerance")
    sat = nreq / cspan
    progress(f"closed loop: {sat:.1f} solves/s")
    out = {
        "metric": "solves/s + HBM GB/s at relres 1e-8 vs plain FP64; p50/p99 solve latency",
        "value": achieved, "unit": "solves/s", "n_gpus": 1, "steps": nreq - warm, "warmup": warm,
        "ms_per_step": (span - first) / (nreq - warm) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"serving loop: {nreq} requests, Poisson arrivals at 200/s (seed 1005); 70% P1 "
                               "finite-element systems from the batch generator, 30% 3D 7-point Dirichlet Laplacians "
                               "with m ~ U{16..100}; tol 1e-6 or 1e-8; 1 right-hand side each; memory-budgeted "
                               "admission, continuous batching, float32 inner + float64 refinement; latency = arrival "
                               "to answer on the host, CSR upload included",
                   "budget_mb": args.serve_budget_mb, "slots": args.serve_slots},
        "p50_ms": float(np.percentile(L, 50)), "p99_ms": float(np.percentile(L, 99)),
        "p50_ms_fe": float(np.percentile(lat[warm:][[r["fe"] for r in reqs[warm:]]] * 1e3, 50)),
        "p50_ms_laplacian": float(np.percentile(lat[warm:][[not r["fe"] for r in reqs[warm:]]] * 1e3, 50)),
        "max_queue": int(qmax),
        "closed_loop_solves_per_s": sat,
        "closed_loop_p50_ms": float(np.percentile(clat * 1e3, 50)),
        "roofline": None,
    }
    if args.serve_small_budget_mb:
        slat, sspan, sq, sbad, _ = run_server(naj, reqs, int(args.serve_small_budget_mb) << 20, args.serve_slots,
                                              False, progress, "small budget")
        if sbad:
            raise SystemExit(f"serve (small budget): {sbad} requests did not converge or missed their tolerance")
        S = slat[warm:] * 1e3
        out["small_budget"] = {"budget_mb": args.serve_small_budget_mb, "p50_ms": float(np.percentile(S, 50)),
                               "p99_ms": float(np.percentile(S, 99)), "max_queue": int(sq),
                               "solves_per_s": (nreq - warm) / (sspan - first)}
    if not args.no_compare:
        # plain float64, one request at a time (a sample of the trace, system built per request as in serving)
        sample = range(warm, min(nreq, warm + args.serve_fp64_sample))
        errs = []
        t0 = time.perf_counter()
        for i in sample:
            r = reqs[i]
            s = r["sys"]
            sm = naj.System(s.rowptr, s.colidx, s.vals)
            x, inf = sm.solve(r["b"], tol=r["tol"], max_iter=20000, hist_cap=0)
            xh = x.cpu().numpy()
            sm.close()
            if i in served:   # the served (mixed) answer against this float64 answer to the same tolerance
                errs.append(float(np.linalg.norm(served[i] - xh) / np.linalg.norm(xh)))
        dt = time.perf_counter() - t0
        out["compare_one_at_a_time"] = {"precision": "fp64", "sampled_requests": len(sample), "seconds": dt,
                                        "solves_per_s": len(sample) / dt,
                                        "rel_err_served_vs_fp64": {"requests": len(errs),
                                                                   "median": float(np.median(errs)) if errs else None,
                                                                   "max": float(np.max(errs)) if errs else None}}
        progress(f"float64 one at a time: {len(sample) / dt:.1f} solves/s")
    return out


def bench_single(args, workload: str, progress, steps: int, warmup: int, precision: str, compare: bool,
                 cpu: bool, sysobj=None) -> dict:
    """One system solved `steps` times (after `warmup` untimed solves) in `precision`; optionally the
    same system in the other precision for the mixed-vs-float64 comparison, and the CPU oracle."""
    import torch
    from paper_2407_03272_amd import naj
    if sysobj is None:
        sysobj = make_workload(workload)
    n, nnz = sysobj.n, sysobj.nnz
    progress(f"workload {sysobj.name}: n={n} nnz={nnz}")
    dev = torch.device("cuda:0")
    jb = args.jblock
    obj = args.stop == "objective"
    if obj:
        if precision != "fp64":
            raise SystemExit("the objective-gap stop is a float64 option")
        compare = False
        fstar = -0.5 * float(np.dot(sysobj.b, sysobj.xstar))
        stop_kw = dict(stop=naj.NAJ_STOP_OBJECTIVE, fstar=fstar)
        tol = 1e-10
    else:
        stop_kw, tol = {}, 1e-8
    sysm = naj.System(sysobj.rowptr, sysobj.colidx, sysobj.vals, device="cuda:0", jblock=jb or None)
    b = torch.as_tensor(sysobj.b).to(dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    mixed = precision == "mixed"
    singular = workload.startswith("chunglu")   # graph Laplacians: answers are defined up to the null space

    def timed(mixed_: bool, steps: int, warmup: int):
        opts = dict(tol=tol, max_iter=20000, precision=naj.NAJ_MIXED if mixed_ else naj.NAJ_FP64,
                    **(stop_kw if not mixed_ else {}))
        for _ in range(warmup):
            sysm.solve(b, out=x, hist_cap=0, **opts)
        torch.cuda.synchronize()
        lat, kms, infos = [], [], []
        t_start = time.perf_counter()
        for _ in range(steps):
            t0 = time.perf_counter()
            _, info = sysm.solve(b, out=x, hist_cap=64 if mixed_ else 0, **opts)
            lat.append(time.perf_counter() - t0)
            kms.append(info.kernel_ms)
            infos.append(info)
            if info.status != 0:
                raise SystemExit(f"solve did not converge: status {info.status}")
        torch.cuda.synchronize()
        total = time.perf_counter() - t_start
        return total, lat, kms, infos

    progress("system created")
    total, lat, kms, infos = timed(mixed, steps, warmup)
    x_main = x.clone()
    progress(f"timed {steps} solves: {total / steps * 1e3:.2f} ms each")
    info = infos[-1]
    sinfo = sysm.info()
    nnz_off = sinfo["offset_nnz"]
    vb = sinfo["value_bytes"]          # 4: the float64 passes read the exact float32 copy of the values
    alg_bytes = solve_bytes(n, nnz, info, mixed, jb, vb=vb)           # CSR int32 yardstick, s_v = vb
    moved_bytes = solve_bytes(n, nnz, info, mixed, jb, nnz_off, vb)  # what the layout reads and writes
    kernel_s = float(np.mean(kms)) / 1e3
    achieved = alg_bytes / kernel_s / 1e9
    solves_s = steps / total
    if mixed:
        per_launch = bytes_per_iteration(n, nnz, s_v=4, s_x=4, jb=jb)
        moved_launch = bytes_per_iteration(n, nnz, s_v=4, s_x=4, jb=jb, nnz_off=nnz_off)
        wl = (f"{sysobj.name}: n={n}, nnz={nnz}; float32 inner accelerated Jacobi with float64 reductions inside "
              f"float64 iterative refinement, x0=0, restart on, K0=2, inner tol 1e-4, final relres <= 1e-8, single solve")
    else:
        per_launch = bytes_per_iteration(n, nnz, s_v=vb, jb=jb)
        moved_launch = bytes_per_iteration(n, nnz, s_v=vb, jb=jb, nnz_off=nnz_off)
        wl = (f"{sysobj.name}: n={n}, nnz={nnz}, float64, x0=0, restart on, K0=2, tol 1e-8, single solve "
              f"(plain FP64 one system at a time)")
        if vb == 4:
            wl += ("; float64 arithmetic and vectors, matrix values read from their float32 copy (every value is "
                   "exact in float32: results bit-identical to 8-byte values)")
    if jb:
        wl += f"; block-diagonal J of eq. (J-blkdiag), blocks of {jb} rows"
    if obj:
        wl = wl.replace("tol 1e-8", "stop on the relative objective gap <= 1e-10 (f* = -<b, x*>/2)")
    line = {
        "metric": "solves/s + HBM GB/s at relres 1e-8 vs plain FP64; p50/p99 solve latency",
        "value": solves_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": total / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": wl, "n": n, "nnz": nnz, "precision": precision, "tol": tol,
                   "iterations": info.iterations, "restarts": info.restarts, "confirmations": info.confirmations,
                   "passes": info.passes, "grid": info.grid, "relres": info.relres,
                   "layout": sinfo["layout"], "offset_slices": sinfo["offset_slices"],
                   "nslices": sinfo["nslices"], "offset_nnz": nnz_off, "value_bytes": vb, "jblock": jb,
                   "stop": args.stop,
                   "objgap": info.objgap if obj else None},
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "kernel_ms": float(np.mean(kms)),
        "gbps_solve": achieved,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if (mixed or jb) else measured_traffic(workload, info.grid, vb),
                     "kernel": "k_pass64 (fused iteration pass, one launch per pass)",
                     "launches_per_solve": info.passes,
                     "algorithmic_bytes_per_launch": per_launch,
                     "layout_bytes_per_launch": moved_launch,
                     "layout_gbps": moved_bytes / kernel_s / 1e9,
                     "layout_frac": moved_bytes / kernel_s / 1e9 / HBM_PEAK_GBS,
                     "mean_launch_us": kernel_s / info.passes * 1e6,
                     "yardstick_note": ("achieved counts the CSR yardstick's bytes: (s_v + 4) per nonzero (int32 "
                                        "columns), int32 row pointers, four vector streams, with s_v the bytes "
                                        f"of a stored value ({4 if mixed else vb}"
                                        + ("; the float64 passes read the values' exact float32 copy" if vb == 4 and not mixed else "")
                                        + "); the layout moves layout_bytes_per_launch (no column indices in "
                                        "column-offset slices); layout_frac is the pass against peak by those bytes")},
    }
    if compare:
        # the same system solved in the other precision, for the mixed-vs-FP64 comparison
        ctot, clat, ckms, cinfos = timed(not mixed, max(3, steps // 2), 1)
        ci = cinfos[-1]
        # the mixed answer against the float64 one (which equals the oracle's in the parity tests); a singular
        # system's answers may differ by a null-space component, so none is stated there
        xm, xf = (x_main, x) if mixed else (x, x_main)
        if singular:
            # answers of a graph Laplacian are defined up to its null space: compare them with the
            # J-weighted mean of every connected component removed (both runs start from x^0 = 0,
            # whose component means the method keeps, so this removes only rounding drift)
            pm = component_mean_free(sysobj.rowptr, sysobj.colidx, sysobj.vals, xm.cpu().numpy())
            pf = component_mean_free(sysobj.rowptr, sysobj.colidx, sysobj.vals, xf.cpu().numpy())
            rel_err = float(np.linalg.norm(pm - pf) / np.linalg.norm(pf))
        else:
            rel_err = float(torch.linalg.vector_norm(xm - xf) / torch.linalg.vector_norm(xf))
        line["compare"] = {"precision": "fp64" if mixed else "mixed", "solves_per_s": len(clat) / ctot,
                           "p50_ms": float(np.percentile(clat, 50) * 1e3),
                           "p99_ms": float(np.percentile(clat, 99) * 1e3),
                           "iterations": ci.iterations, "confirmations": ci.confirmations, "relres": ci.relres,
                           "rel_err_mixed_vs_fp64": rel_err,
                           "rel_err_definition": ("2-norm over 2-norm after removing each connected component's "
                                                  "J-weighted mean" if singular else "2-norm over 2-norm"),
                           "gbps_solve": solve_bytes(n, nnz, ci, not mixed, jb) / (float(np.mean(ckms)) / 1e3) / 1e9}
    it = info.iterations
    if cpu:
        progress("cpu baseline")
        its_fp64 = info.iterations if not mixed else line.get("compare", {}).get("iterations", info.iterations)
        line["cpu_baseline"] = cpu_baseline(sysobj, its_fp64, args.cpu_sample_iters, jb or None,
                                            dict(stop="objective", fstar=stop_kw["fstar"]) if obj else None,
                                            progress)
    sysm.close()
    return line



def _sub(line: dict) -> dict:
    """A workload's result as a sub-object of the default line (without the keys the top line carries)."""
    return {k: v for k, v in line.items()
            if k not in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data")}


MALL_BYTES = 256 << 20      # MI355X Infinity Cache


def residency(rf: dict) -> str:
    """Whether a pass's own bytes fit the MALL, which can then serve part of them between passes."""
    mib = rf["layout_bytes_per_launch"] / (1 << 20)
    if rf["layout_bytes_per_launch"] <= MALL_BYTES:
        return (f"MALL-resident: the pass moves about {mib:.0f} MiB, under the 256 MiB MALL, so part of its "
                "bytes may come from the MALL rather than HBM")
    return f"beyond the MALL: about {mib:.0f} MiB moved per pass"


def bench_default(args, progress) -> dict:
    """The default run.  Top level: the 128^3 Laplacian in float64, one solve per step (value, latency,
    the fused pass's roofline, the mixed-precision comparison, the CPU oracle), and the measured copy
    bandwidth.  Sub-results, each with its own fixed step counts: the 64x64 Poisson system in float64
    (against mixed and the CPU oracle), 160^3 and 192^3 in float64 (with 4-byte values the 160^3 pass
    fits the 256 MiB MALL, the 192^3 pass does not), the Chung-Lu graph Laplacian n = 2^22 in mixed precision against float64, the
    512-system finite-element batch (mixed batch against float64 batch and float64 one system at a
    time), and the serving loop (p50/p99 latency, offered and saturated solves/s, float64 one request
    at a time)."""
    import copy
    t_start = time.perf_counter()
    line = bench_single(args, "laplace3d_128", progress, args.steps, args.warmup, "fp64", not args.no_compare,
                        not args.no_cpu_baseline)
    if line["config"].get("value_bytes") == 4:
        # the same solve with the 8-byte values (NAJ_VALUES32=0, its own 256 x 3 launch): the same answer
        # bit for bit, for the comparison with the 4-byte reads the value above uses
        os.environ["NAJ_VALUES32"] = "0"
        try:
            v8 = bench_single(args, "laplace3d_128", progress, max(3, args.steps // 2), 1, "fp64", False, False)
        finally:
            del os.environ["NAJ_VALUES32"]
        line["values8"] = {"solves_per_s": v8["value"], "ms_per_step": v8["ms_per_step"],
                           "mean_launch_us": v8["roofline"]["mean_launch_us"], "grid": v8["config"]["grid"],
                           "layout_bytes_per_launch": v8["roofline"]["layout_bytes_per_launch"],
                           "layout_frac": v8["roofline"]["layout_frac"], "frac": v8["roofline"]["frac"],
                           "iterations": v8["config"]["iterations"],
                           "note": "8-byte matrix values (NAJ_VALUES32=0); every other setting as in the value"}
    ab = attainable_bandwidth(progress)
    line["attainable_bandwidth"] = ab
    rf = line["roofline"]
    rf["attainable_gbps"] = ab["best_gbps"]
    rf["frac_of_attainable"] = rf["achieved"] / ab["best_gbps"]
    rf["layout_frac_of_attainable"] = rf["layout_gbps"] / ab["best_gbps"]
    rf["residency"] = residency(rf)
    subs = {}
    # the small configuration: 64x64 Poisson in float64 beside the CPU oracle (all host threads), and mixed
    subs["poisson2d_64"] = _sub(bench_single(args, "poisson2d_64", progress, 50, 5, "fp64", True,
                                             not args.no_cpu_baseline))
    progress(f"64x64 done at {time.perf_counter() - t_start:.0f} s")
    for w in ("laplace3d_160", "laplace3d_192"):
        subs[w] = _sub(bench_single(args, w, progress, 3, 1, "fp64", True, False))
        subs[w]["roofline"]["residency"] = residency(subs[w]["roofline"])
        progress(f"{w} done at {time.perf_counter() - t_start:.0f} s")
    subs["chunglu_4m"] = _sub(bench_single(args, "chunglu_4m", progress, 3, 1, "mixed", True, False))
    progress(f"Chung-Lu done at {time.perf_counter() - t_start:.0f} s")
    a2 = copy.copy(args)
    a2.steps, a2.warmup, a2.precision = 2, 1, "mixed"
    fe = bench_fe_batch(a2, progress)
    subs["fe_batch"] = _sub(fe)
    progress(f"batch done at {time.perf_counter() - t_start:.0f} s")
    sv = bench_serve(args, progress)
    subs["serve"] = _sub(sv)
    progress(f"serving done at {time.perf_counter() - t_start:.0f} s")
    line["workloads"] = subs
    one_fe = fe.get("compare_one_at_a_time", {}).get("solves_per_s_est")
    one_sv = sv.get("compare_one_at_a_time", {}).get("solves_per_s")
    line["comparisons"] = {
        "batched_mixed_solves_per_s": fe["value"],
        "batched_fp64_solves_per_s": fe.get("compare_batch", {}).get("solves_per_s"),
        "fp64_one_at_a_time_solves_per_s_batch_systems": one_fe,
        "batched_mixed_over_fp64_one_at_a_time": fe["value"] / one_fe if one_fe else None,
        "served_mixed_solves_per_s_offered_200": sv["value"],
        "served_mixed_solves_per_s_saturated": sv["closed_loop_solves_per_s"],
        "served_p50_ms": sv["p50_ms"], "served_p99_ms": sv["p99_ms"],
        "fp64_one_at_a_time_solves_per_s_trace": one_sv,
        "served_saturated_over_fp64_one_at_a_time": sv["closed_loop_solves_per_s"] / one_sv if one_sv else None,
    }
    line["bench_seconds"] = time.perf_counter() - t_start
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="laplace3d_128")
    ap.add_argument("--cpu-sample-iters", type=int, default=200)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-compare", action="store_true", help="skip the second-precision comparison solves")
    ap.add_argument("--nsys", type=int, default=512, help="systems in the fe_batch workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stop", choices=["relres", "objective"], default="relres",
                    help="single float64 solves: stop on the relative residual (tol 1e-8) or on the paper's "
                         "relative objective gap (tol 1e-10, f* = -<b, x*>/2 from the generator's x*)")
    ap.add_argument("--jblock", type=int, default=0,
                    help="single-solve workloads: block-diagonal J of eq. (J-blkdiag) with blocks of this many rows")
    ap.add_argument("--serve-requests", type=int, default=2200, help="requests in the serve workload trace")
    ap.add_argument("--serve-budget-mb", type=int, default=8192, help="serve workload memory budget")
    ap.add_argument("--serve-small-budget-mb", type=int, default=512, help="second serve run with this budget (0: none)")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-fp64-sample", type=int, default=200)
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the beyond-MALL, Chung-Lu, batch and serving sub-results")
    ap.add_argument("--pmc-sample", action="store_true",
                    help="run only a 1 GiB torch copy (counter calibration) and a 50-iteration solve, for rocprofv3 --pmc")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(a single system's solve runs on one device)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_03272_amd import naj

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.workload == "serve":
        print(json.dumps(bench_serve(args, progress)), flush=True)
        return
    if args.workload == "fe_batch":
        if args.precision == "fp64" and "--precision" not in sys.argv:
            args.precision = "mixed"
        print(json.dumps(bench_fe_batch(args, progress)), flush=True)
        return
    if args.pmc_sample:
        # counter calibration: the library's probe kernel reads 1 GiB (mode 0) and copies 1 GiB (mode 1),
        # two launches each (one untimed, one timed); then 50 iterations of the workload's solve
        sysobj = make_workload(args.workload)
        dev = torch.device("cuda:0")
        cal = [naj.bandwidth_probe(m, 1 << 30, 1) for m in (0, 1)]
        torch.cuda.synchronize()
        sysm = naj.System(sysobj.rowptr, sysobj.colidx, sysobj.vals, device="cuda:0")
        b = torch.as_tensor(sysobj.b).to(dev)
        prec = naj.NAJ_MIXED if args.precision == "mixed" else naj.NAJ_FP64
        _, info = sysm.solve(b, hist_cap=0, tol=1e-30, max_iter=50, precision=prec,
                             **({"max_refine": 1} if prec == naj.NAJ_MIXED else {}))
        print(json.dumps({"pmc_sample": True, "probe_read_bytes": 1 << 30, "probe_copy_bytes_each_way": 1 << 30,
                          "probe": cal, "passes": info.passes, "info": sysm.info()}))
        return
    if args.workload == "laplace3d_128" and not args.no_extras and args.precision == "fp64" and not args.jblock \
            and args.stop == "relres":
        print(json.dumps(bench_default(args, progress)), flush=True)
        return
    line = bench_single(args, args.workload, progress, args.steps, args.warmup, args.precision,
                        not args.no_compare, not args.no_cpu_baseline)
    print(json.dumps(line), flush=True)

if __name__ == "__main__":
    main()
