#!/usr/bin/env python
"""Throughput of the AZ least-squares RBF solver on one MI355X.

Workload (default): 1D batched AZ in FP64, 65536 Gaussian RBF centres on the
periodic box [-1, 1), eps*h = 0.5, s = 2, domain [-0.5, 0.5] (M = 65537
collocation rows), 64 right-hand sides (seeded random trigonometric sums),
one shared low-rank factor (sketch width k = 32).

One step = the whole hot path on one batch: plan (index list, spectra, B^+
weights), factor (sketch, TSQR, Jacobi SVD), the solve of all right-hand
sides (Algorithm 1 plus one refinement pass) and their residuals.  The
right-hand sides are resident in HBM before the timed region.  ``value`` is
right-hand sides solved per second whose residual ||Ax - b||/||b|| is at most
1e-10.

Also reported: the plain per-problem rate (each right-hand side its own
plan + factor + solve), the rate with a resident factor and one right-hand
side per call, the roofline of the kernel with the largest share of GPU time
(HIP events around each launch on its own stream, algorithmic bytes or flops
per launch) and of the FFT passes together, a served-stream comparison
(continuous batching with resident factors against plain FIFO solves on a
reduced mixed 1D/2D request stream, with p50/p99 latency), and the CPU
oracle timed on a bounded sample of the same family.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AZ solves/sec at residual <=1e-10 (batched/served vs plain); FFT-pass HBM GB/s"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(n=4096, nrhs=64):
    """The oracle (dense truncated SVD) on the same 1D family at n centres."""
    import numpy as np
    import workloads as W
    from oracle import dense, lstsq
    prob = W.config_c2(n=n, nrhs=nrhs)
    t0 = time.perf_counter()
    A, idx, pts, bpts = dense.system_matrix(prob)
    B = dense.rhs(prob, pts, bpts)
    t1 = time.perf_counter()
    svd = lstsq.tsvd(A)
    t2 = time.perf_counter()
    X, _ = lstsq.tsvd_solve(A, B, 1e-12, svd=svd)
    t3 = time.perf_counter()
    rel = np.linalg.norm(A @ X - B, axis=0) / np.linalg.norm(B, axis=0)
    threads = None
    try:
        import threadpoolctl
        threads = max(i.get("num_threads", 0) for i in threadpoolctl.threadpool_info())
    except Exception:
        pass
    cores = threads or len(os.sched_getaffinity(0))
    total = t3 - t0
    return {
        "value": nrhs / total, "unit": "solves/s", "cores": cores, "kind": "oracle",
        "sample": f"1D family at N={n} (M={A.shape[0]}), {nrhs} RHS: dense A assembly "
                  f"{t1 - t0:.2f}s + LAPACK gesdd {t2 - t1:.2f}s + back-substitution {t3 - t2:.3f}s; "
                  f"max relres {rel.max():.1e}",
        "extrapolated_full_size": {"value": nrhs / (total * (65536 / n) ** 3), "unit": "solves/s",
                                   "rule": "dense SVD cost O(M N^2) scaled from the sample"},
    }


def _traffic(kernel):
    """HBM bytes per launch from the stored rocprofv3 FETCH_SIZE / WRITE_SIZE
    passes (calibrated against a copy of known size), if they were taken on
    the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2308_14490_amd.traffic import source_hash
    if t.get("source_hash") != source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def by_kernel(recs):
    """Per-launch records grouped by kernel: the leaf and tree levels of the
    TSQR (and of the Q formation) are launches of one kernel, as in a
    rocprofv3 kernel trace."""
    out = {}
    for r in recs:
        name = r["name"].replace(" (tree)", "")
        e = out.setdefault(name, {"name": name, "calls": 0, "ms": 0.0, "max_ms": 0.0, "bytes": 0.0, "flops": 0.0})
        e["calls"] += r["calls"]
        e["ms"] += r["ms"]
        e["max_ms"] = max(e["max_ms"], r.get("max_ms", 0.0))
        e["bytes"] += r["bytes"]
        e["flops"] += r.get("flops", 0.0)
    return list(out.values())


def roofline_of(r, total_ms):
    """Roofline entry of one kernel from the per-launch profile record."""
    avg_ms = r["ms"] / r["calls"]
    flops = r.get("flops", 0.0)
    if flops > 0 and flops / max(r["bytes"], 1.0) > FP64_PEAK_TFS * 1e3 / HBM_PEAK_GBS:
        achieved = flops / r["calls"] / (avg_ms * 1e-3) / 1e12
        out = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
               "frac": round(achieved / FP64_PEAK_TFS, 4)}
    else:
        achieved = r["bytes"] / r["calls"] / (avg_ms * 1e-3) / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(achieved / HBM_PEAK_GBS, 4)}
    out.update({"traffic": _traffic(r["name"]), "kernel": r["name"], "avg_us": round(avg_ms * 1e3, 2),
                "bytes_per_launch": r["bytes"] / r["calls"], "share_of_gpu_time": round(r["ms"] / total_ms, 3)})
    return out


def served_vs_plain(count, seed, sides, log_fn, modes=("plain", "closed", "open"), rate=None):
    """Mixed stream (70% 1D N = 2^10..2^16, 30% 2D approximation on disks
    and stars of the given sides): plain FIFO per-problem solves against the
    continuous-batching server, both closed-loop (all requests queued at the
    start), then the server open-loop (Poisson arrivals at `rate`, by default
    twice the plain request rate).  `modes` selects the parts to run."""
    import torch
    import workloads as W
    from paper_2308_14490_amd import serve
    be = serve.GpuBackend()
    free, total = torch.cuda.mem_get_info()
    budget = int(min(free * 0.8, 200 << 30))
    reqs = W.served_stream(count=count, seed=seed, rate=1e9, sides=sides)
    for r in reqs:
        r.arrival = 0.0
    last = [time.perf_counter()]
    dims = {r.rid: r.problem.dim for r in reqs}

    def by_dim(res):
        """p50 / p99 latency of the 1D and of the 2D requests separately."""
        import numpy as np
        out_d = {}
        for d in (1, 2):
            lat = [(r.done - r.arrival) * 1e3 for r in res.values() if dims[r.rid] == d]
            if lat:
                out_d[f"{d}d"] = {"requests": len(lat), "p50_ms": float(np.percentile(lat, 50)),
                                  "p99_ms": float(np.percentile(lat, 99))}
        return out_d

    def progress(done, tot):
        now = time.perf_counter()
        if done == tot or now - last[0] > 20.0:
            last[0] = now
            log_fn(f"  {done}/{tot} requests done")
    # warm the kernels of every size once
    warm = {}
    for r in reqs:
        key = (r.problem.dim, r.problem.n)
        if key not in warm:
            warm[key] = r
    serve.run_plain(be, list(warm.values()))
    torch.cuda.synchronize()
    out = {"requests": count, "seed": seed, "sides_2d": list(sides), "exps_1d": [10, 16], "budget_bytes": budget}
    if "plain" in modes:
        res = serve.run_plain(be, reqs, progress=progress)
        plain = dict(serve.summarize(res), by_dim=by_dim(res))
        log_fn(f"served stream: plain {plain['solves_per_s']:.1f} solves/s, p50 {plain['p50_ms']:.1f} ms")
        out["plain"] = plain
    if "closed" in modes:
        srv = serve.Server(be, budget)
        res = srv.run(reqs, progress=progress)
        closed = dict(serve.summarize(res), by_dim=by_dim(res))
        srv.close()
        log_fn(f"served stream: served closed-loop {closed['solves_per_s']:.1f} solves/s")
        out["served_closed_loop"] = closed
        if "plain" in out:
            out["speedup_closed_loop"] = round(closed["solves_per_s"] / out["plain"]["solves_per_s"], 3)
    if "open" in modes:
        if rate is None:
            rate = 2.0 * out["plain"]["requests"] / out["plain"]["makespan_s"]
        open_reqs = W.served_stream(count=count, seed=seed, rate=rate, sides=sides)
        srv = serve.Server(be, budget)
        res = srv.run(open_reqs, progress=progress)
        openl = dict(serve.summarize(res), by_dim=by_dim(res))
        ticks = len(srv.ticks)
        srv.close()
        log_fn(f"served stream: open-loop at {rate:.1f} req/s: p50 {openl['p50_ms']:.1f} ms "
               f"p99 {openl['p99_ms']:.1f} ms")
        out["served_open_loop"] = dict(openl, rate_req_per_s=round(rate, 2), groups=ticks)
    be.close()
    return out


def wide_2d(log_fn, n=128):
    """The 2D approximation workload at full size (disk of radius 0.8, n x n
    centres, eps*h = 0.5): factor (sketch, BCGS2 QR, block Jacobi SVD on the
    matrix cores) and one solve, with the matrix-core kernels' utilisation."""
    import torch
    import workloads as W
    from paper_2308_14490_amd import azrbf, problems
    prob = W.config_c3a(n)
    p = problems.plan_for(prob)
    B = problems.rhs_for(p, prob)
    torch.cuda.synchronize()
    azrbf.profile_enable(True)
    t0 = time.perf_counter()
    azrbf.factor(p)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    X, rel = azrbf.solve(p, B)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    kern = azrbf.profile_report()
    azrbf.profile_enable(False)
    inf = p.info()
    p.destroy()
    mfma = {}
    for r in kern:
        if r.get("flops", 0) > 0 and r["ms"] > 0:
            tf = r["flops"] / (r["ms"] * 1e-3) / 1e12
            mfma[r["name"]] = {"calls": r["calls"], "ms": round(r["ms"], 2), "TFLOPs": round(tf, 2),
                               "frac_of_fp64_peak": round(tf / FP64_PEAK_TFS, 4)}
    tot_f = sum(r.get("flops", 0) for r in kern)
    tot_ms = sum(r["ms"] for r in kern if r.get("flops", 0) > 0)
    out = {"workload": f"2D disk R=0.8, {n}x{n} centres, eps*h=0.5, M={inf['M']}",
           "k": inf["k"], "rank": inf["rank"], "sweeps": inf["sweeps"], "factor_s": round(t1 - t0, 3),
           "solve_s": round(t2 - t1, 4), "relres": float(rel.max()), "mfma_kernels": mfma,
           "mfma_TFLOPs_overall": round(tot_f / (tot_ms * 1e-3) / 1e12, 2) if tot_ms else None}
    log_fn(f"2D n={n}: factor {out['factor_s']} s (k {inf['k']}, rank {inf['rank']}), relres {out['relres']:.2e}, "
           f"matrix-core kernels {out['mfma_TFLOPs_overall']} TF/s")
    return out


def beyond_cache(log_fn, nvec=512, pairs_per_launch=256):
    """The FFT passes with every pass's working set past the 256 MB Infinity
    Cache: A, Z* and A Z* on nvec vectors at N = 65536 with all of them in
    one launch per pass (each pass reads and writes 0.5-1.1 GB), per-launch
    HIP-event timing.  Rates here are HBM rates."""
    import torch
    import workloads as W
    from paper_2308_14490_amd import azrbf, problems
    prob = W.config_c2(65536, 1)
    key = "e1_256x256_s2"
    saved = azrbf.tune_table()
    shape = saved.get(key, (16, 4, 0))
    azrbf.tune_load({key: (shape[0], shape[1], pairs_per_launch)})
    p = problems.plan_for(prob)
    X = azrbf.gaussian(7, p.N, nvec)
    Y = azrbf.apply_A(p, X)
    Z = azrbf.apply_Zstar(p, Y)
    azrbf.apply_AZstar(p, Y, Y, alpha=-1.0, beta=1.0)
    torch.cuda.synchronize()
    azrbf.profile_enable(True)
    for _ in range(2):
        azrbf.apply_A(p, X, Y)
        azrbf.apply_Zstar(p, Y, Z)
        azrbf.apply_AZstar(p, Y, Y, alpha=-1.0, beta=1.0)
    torch.cuda.synchronize()
    rep = azrbf.profile_report()
    azrbf.profile_enable(False)
    p.destroy()
    del X, Y, Z
    azrbf.tune_load({key: shape})
    azrbf.release_cached_memory()
    fft = [r for r in rep if r["name"].startswith(("col_", "row_"))]
    b = sum(r["bytes"] for r in fft)
    ms = sum(r["ms"] for r in fft)
    kern = {r["name"]: {"calls": r["calls"], "avg_us": round(r["ms"] / r["calls"] * 1e3, 1),
                        "MB_per_launch": round(r["bytes"] / r["calls"] / 1e6, 1),
                        "GBps": round(r["bytes"] / (r["ms"] * 1e-3) / 1e9, 1),
                        "frac": round(r["bytes"] / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)} for r in fft}
    out = {"workload": f"apply_A, apply_Zstar, apply_AZstar on {nvec} vectors, N=65536, s=2, "
                       f"{pairs_per_launch} vector pairs per launch",
           "achieved": round(b / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "kernels": kern}
    log_fn(f"FFT passes past the cache ({nvec} vectors): {out['achieved']} GB/s ({out['frac']})")
    return out


def bvp_2d(log_fn, n=256, nrhs=64):
    """The 2D Poisson workload at full size (star 0.7 + 0.1 cos 5t, n x n
    centres, weak Dirichlet rows): factor time, and solves per second with the
    factor resident, one right-hand side per call against nrhs per call (the
    workload's manufactured data plus seeded random-trig interior and
    boundary data), plus the plain per-problem rate (factor + one solve)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2308_14490_amd import azrbf, problems
    prob = W.config_c4(n)
    prob.rhs = prob.rhs + [W.trig_sum_2d(3000 + i) for i in range(nrhs - 1)]
    prob.bnd = prob.bnd + [W.trig_sum_2d(5000 + i) for i in range(nrhs - 1)]
    p = problems.plan_for(prob)
    B = problems.rhs_for(p, prob)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    azrbf.factor(p)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    X1, r1 = azrbf.solve(p, B[:1].contiguous())
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    reps = 4
    for _ in range(reps):
        X1, r1 = azrbf.solve(p, B[:1].contiguous())
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    X, rel = azrbf.solve(p, B)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(2):
        X, rel = azrbf.solve(p, B)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    inf = p.info()
    rels = rel.cpu().numpy()
    good_b = int(np.sum(rels <= 1e-10))
    good_1 = int(float(r1.max()) <= 1e-10)
    one = (t3 - t2) / reps
    out = {"workload": f"2D Poisson star R=0.7+0.1cos5t, {n}x{n} centres, eps*h=0.5, M={inf['M']}, Mb={inf['Mb']}, "
                       f"refine={p._prob.refine}",
           "k": inf["k"], "rank": inf["rank"], "sweeps": inf["sweeps"], "factor_s": round(t1 - t0, 3),
           "solve_1rhs_s": round(one, 4), "solve_batch_s": round((t5 - t4) / 2, 4), "nrhs_batch": nrhs,
           "relres_workload_rhs": float(rels[0]), "max_relres": float(rels.max()),
           "solves_per_s": {"plain_per_problem": round(good_1 / (t1 - t0 + one), 3),
                            "plain_resident_factor": round(good_1 / one, 2),
                            "batched_resident_factor": round(good_b / ((t5 - t4) / 2), 2)}}
    p.destroy()
    azrbf.release_cached_memory()
    log_fn(f"2D Poisson n={n}: factor {out['factor_s']} s (k {inf['k']}, rank {inf['rank']}), "
           f"relres {out['relres_workload_rhs']:.2e}, solves/s {out['solves_per_s']}")
    return out


def million_1d(log_fn, n=1 << 20, nrhs=64):
    """The 1D family at N = 2^20 centres (M = 2^20 + 1; the paper solves up to
    N = 10^6): plan + factor + solve of one right-hand side, and of nrhs."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2308_14490_amd import azrbf, problems
    prob = W.family_1d(n, nrhs)
    p = problems.plan_for(prob)
    B = problems.rhs_for(p, prob)
    X, rel = azrbf.solve(p, B)         # warm-up: first launches at this size
    torch.cuda.synchronize()
    p.destroy()
    out = {"workload": f"1D N={n}, M={p.M}, eps*h=0.5, s=2, random-trig RHS, k=32"}
    for cnt in (1, nrhs):
        Bc = B[:cnt].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = problems.plan_for(prob)
        X, rel = azrbf.solve(p, Bc)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        good = int((rel <= 1e-10).sum())
        out[f"plan_factor_solve_{cnt}rhs_s"] = round(dt, 5)
        out[f"solves_per_s_{cnt}rhs"] = round(good / dt, 1)
        out[f"max_relres_{cnt}rhs"] = float(rel.max())
        p.destroy()
    azrbf.release_cached_memory()
    log_fn(f"1D N={n}: plan+factor+solve 1 RHS {out['plan_factor_solve_1rhs_s'] * 1e3:.1f} ms, "
           f"{nrhs} RHS {out[f'plan_factor_solve_{nrhs}rhs_s'] * 1e3:.1f} ms")
    return out


def transform_paths(log_fn, nvec=64):
    """apply_A followed by apply_Z* on nvec vectors at about a million
    centres through the three transform paths: the power-of-two engine
    (N = 2^20), mixed radix (N = 10^6 = 2^6 5^6) and Bluestein (N = 999983,
    a prime), ms per pair of applications (best of three)."""
    import torch
    import workloads as W
    from paper_2308_14490_amd import azrbf, problems
    out = {"workload": f"apply_A then apply_Zstar on {nvec} vectors, 1D family, s=2"}
    for name, n in (("engine_2^20", 1 << 20), ("mixed_radix_10^6", 10 ** 6), ("bluestein_999983", 999983)):
        p = problems.plan_for(W.family_1d(n, 1))
        X = azrbf.gaussian(3, p.N, nvec)
        Y = azrbf.apply_A(p, X)
        Z = azrbf.apply_Zstar(p, Y)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(3):
            t0 = time.perf_counter()
            azrbf.apply_A(p, X, Y)
            azrbf.apply_Zstar(p, Y, Z)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        out[name] = {"N": n, "ms": round(best * 1e3, 2)}
        p.destroy()
        del X, Y, Z
    azrbf.release_cached_memory()
    log_fn("transform paths: " + ", ".join(f"{k} {v['ms']} ms" for k, v in out.items() if isinstance(v, dict)))
    return out


def flower_paper_size(log_fn):
    """Section 6.3's last experiment at the paper's size: Helmholtz on the
    flower with a hole, 100 x 100 centres (mixed radix), 200 Neumann and 100
    Dirichlet points, the paper's source and homogeneous data: plan + factor
    + solve time (the paper's Matlab AZ took 87 s on a laptop)."""
    import torch
    import workloads as W
    from paper_2308_14490_amd import azrbf, problems
    prob = W.config_flower(100)
    p = problems.plan_for(prob)
    B = problems.rhs_for(p, prob)
    torch.cuda.synchronize()
    p.destroy()
    t0 = time.perf_counter()
    p = problems.plan_for(prob)
    X, rel = azrbf.solve(p, B)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    inf = p.info()
    out = {"workload": f"flower r=0.69+0.1cos5t minus a circle of radius 0.1, 100x100 centres, s=2, "
                       f"M={inf['M']}, Mb={inf['Mb']} (200 Neumann, 100 Dirichlet), Helmholtz k^2=4",
           "rows": inf["M"] + inf["Mb"], "cols": inf["N"], "k": inf["k"], "rank": inf["rank"],
           "plan_factor_solve_s": round(dt, 3), "relres": float(rel.max()),
           "coef_norm": float(X.norm())}
    p.destroy()
    azrbf.release_cached_memory()
    log_fn(f"flower 100x100: {out['plan_factor_solve_s']} s, relres {out['relres']:.2e}")
    return out


def copies_1d(log_fn, copies=4096, plain=64):
    """The 256-centre 1D problem (eps*h = 0.5, f = e^x sin 7x + x^2) solved for
    `copies` right-hand sides at once on one plan (one launch sequence for all
    of them) against the plain per-problem solve (plan + factor + solve per
    copy), both gated on the residual."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2308_14490_amd import azrbf, problems
    prob = W.config_c1a(256)
    p = problems.plan_for(prob)
    b = problems.rhs_for(p, prob)
    B = b.expand(copies, -1).contiguous()
    X, rel = azrbf.solve(p, B)
    torch.cuda.synchronize()
    p.destroy()
    reps = 3
    rels = torch.empty((reps, copies), dtype=torch.float64, device=B.device)
    t0 = time.perf_counter()
    for i in range(reps):
        p = problems.plan_for(prob)
        azrbf.solve(p, B, X, rels[i])
        p.destroy()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rp = torch.empty((plain, 1), dtype=torch.float64, device=B.device)
    Xp = torch.empty((1, p.N), dtype=torch.float64, device=B.device)
    t2 = time.perf_counter()
    for i in range(plain):
        q = problems.plan_for(prob)
        azrbf.solve(q, b, Xp, rp[i])
        q.destroy()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    out = {"workload": f"1D N=256, eps*h=0.5, M=257, f=e^x sin7x+x^2; {copies} copies per call",
           "batched_per_problem": round(int((rels <= 1e-10).sum()) / (t1 - t0), 1),
           "plain_per_problem": round(int((rp <= 1e-10).sum()) / (t3 - t2), 1),
           "max_relres": float(rels.max())}
    log_fn(f"1D N=256 copies: batched {out['batched_per_problem']}/s, plain {out['plain_per_problem']}/s")
    return out


def uneven_1d(log_fn, count=256, seed=77, reps=3):
    """Many small 1D problems of uneven sizes with resident factors, the
    per-request work of a serving loop: N = 2^10 .. 2^13, s = 2 or 3,
    eps*h in [0.48, 0.52], seeded intervals inside [-0.7, 0.7], 1..16
    random-trig right-hand sides each.  Solved one plan after another
    (azrbf_solve), on four streams (azrbf_solve_many) and in one grouped call
    (azrbf_solve_batched); every mode counts only right-hand sides with a
    residual <= 1e-10.  The cold passes make new plans each time (plan +
    factor + solve; the grouped call factors them together)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2308_14490_amd import azrbf, problems
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(count):
        n = int(2 ** rng.integers(10, 14))
        s = int(rng.integers(2, 4))
        eh = float(rng.uniform(0.48, 0.52))
        c = float(rng.uniform(-0.2, 0.2))
        w = float(rng.uniform(0.35, 0.5))
        nr = int(rng.integers(1, 17))
        probs.append(W.Problem(f"u{i}", 1, n, s, 1.0, eh, W.interval(c - w, c + w),
                               [W.trig_sum_1d(10000 * seed + 32 * i + j) for j in range(nr)], k=32))
    plans = [problems.plan_for(p) for p in probs]
    Bs = [problems.rhs_for(pl, p) for pl, p in zip(plans, probs)]
    for pl in plans:
        azrbf.factor(pl)
    nrhs = sum(B.shape[0] for B in Bs)
    Xs = [torch.empty((B.shape[0], pl.N), dtype=torch.float64, device=B.device) for pl, B in zip(plans, Bs)]
    rels = [torch.empty(B.shape[0], dtype=torch.float64, device=B.device) for B in Bs]

    def good():
        # one device-side gather of this pass's residuals (no host wait); counted after the timing
        return torch.cat(rels)

    def plain():
        for pl, B, X, r in zip(plans, Bs, Xs, rels):
            azrbf.solve(pl, B, X, r)

    def many():
        azrbf.solve_many(plans, Bs, Xs)

    def grouped():
        azrbf.solve_batched(plans, Bs, Xs, rels)

    out = {"workload": f"{count} 1D problems, N = 2^10..2^13, s = 2..3, eps*h 0.48..0.52, seeded intervals, "
                       f"1..16 RHS each ({nrhs} in all), factors resident",
           "problems": count, "rhs": nrhs}
    for name, fn in (("plain", plain), ("solve_many", many), ("grouped", grouped)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        passes = []
        for _ in range(reps):
            fn()
            if name != "solve_many":
                passes.append(good())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if name == "solve_many":     # solve_many returns its own residual arrays: count them once more
            _, rr = azrbf.solve_many(plans, Bs, Xs)
            torch.cuda.synchronize()
            ok = reps * sum(int((r <= 1e-10).sum()) for r in rr)
        else:
            ok = int(sum(int((p <= 1e-10).sum()) for p in passes))
        out[name] = {"solves_per_s": round(ok / dt, 1), "problems_per_s": round(reps * count / dt, 1),
                     "ms_per_pass": round(dt / reps * 1e3, 3)}
        log_fn(f"uneven 1D {name}: {out[name]}")
    # cold: new plans every pass (plan + factor + solve); grouped factors them together
    def cold(mode):
        ps = [problems.plan_for(p) for p in probs]
        if mode == "plain":
            for pl, B, X, r in zip(ps, Bs, Xs, rels):
                azrbf.solve(pl, B, X, r)
            return ps, rels
        if mode == "solve_many":
            return ps, azrbf.solve_many(ps, Bs, Xs)[1]
        azrbf.solve_batched(ps, Bs, Xs, rels)
        return ps, rels
    for name in ("plain", "solve_many", "grouped"):
        for pl in cold(name)[0]:
            pl.destroy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ps, rr = cold(name)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = sum(int((r <= 1e-10).sum()) for r in rr)
        for pl in ps:
            pl.destroy()
        out["cold_" + name] = {"ms_per_pass": round(dt * 1e3, 2), "problems_per_s": round(count / dt, 1),
                               "rhs_good": ok}
        log_fn(f"uneven 1D cold {name}: {out['cold_' + name]}")
    out["grouped_over_plain"] = round(out["grouped"]["solves_per_s"] / out["plain"]["solves_per_s"], 2)
    out["grouped_over_solve_many"] = round(out["grouped"]["solves_per_s"] / out["solve_many"]["solves_per_s"], 2)
    for pl in plans:
        pl.destroy()
    azrbf.release_cached_memory()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--plain", type=int, default=8, help="right-hand sides timed in the plain modes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=4096)
    ap.add_argument("--no-served", action="store_true", help="skip the served-stream comparison")
    ap.add_argument("--no-2d", action="store_true", help="skip the full-size 2D factorisation")
    ap.add_argument("--retune", action="store_true", help="search the tile shapes instead of loading the table")
    ap.add_argument("--calibrate", action="store_true",
                    help="after the steps, run an elementwise kernel of known size (1 GiB read, 1 GiB written) "
                         "for hardware-counter calibration")
    ap.add_argument("--serve-count", type=int, default=48)
    ap.add_argument("--serve-sides", default="64", help="2D grid sides of the served stream, comma-separated")
    ap.add_argument("--served-only", action="store_true",
                    help="run only the served-stream comparison and print its JSON")
    ap.add_argument("--serve-modes", default="plain,closed,open")
    ap.add_argument("--serve-rate", type=float, default=None, help="open-loop arrival rate (req/s)")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + steps only (for rocprofv3 runs)")
    ap.add_argument("--uneven-only", action="store_true",
                    help="run only the uneven-problems comparison (plain, solve_many, grouped) and print its JSON")
    ap.add_argument("--only-2d", action="store_true",
                    help="run only the full-size 2D factorisation and solve, print its figures as JSON "
                         "(for rocprofv3 runs of the wide-sketch stage)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import workloads as W
    from paper_2308_14490_amd import azrbf, problems

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.only_2d:
        print(json.dumps(wide_2d(log)), flush=True)
        return 0
    if args.uneven_only:
        print(json.dumps(uneven_1d(log)), flush=True)
        return 0
    sides = tuple(int(v) for v in args.serve_sides.split(","))
    if args.served_only:
        azrbf.tune_load_file(os.path.join(ROOT, "paper_2308_14490_amd", "tune_mi355x.json"))
        print(json.dumps(served_vs_plain(args.serve_count, 2024, sides, log, tuple(args.serve_modes.split(",")),
                                         args.serve_rate)), flush=True)
        return 0
    prob = W.config_c2(n=args.n, nrhs=args.nrhs)
    mask = azrbf.make_mask(1, prob.n, prob.s, prob.T, prob.domain.contains)
    p0 = problems.plan_for(prob)
    B = problems.rhs_for(p0, prob, device=dev).contiguous()
    # right-hand sides stored with a leading dimension rounded up to 16 doubles
    # (whole 128-byte lines per column, as the library's own buffers; the values
    # are the same, only the column stride differs)
    ldb = (B.shape[1] + 15) // 16 * 16
    Bp = torch.zeros((B.shape[0], ldb), dtype=torch.float64, device=dev)
    Bp[:, :B.shape[1]] = B
    B = Bp[:, :B.shape[1]]
    M, k = p0.M, p0.k
    # tile shapes of the FFT engine for this operator and batch: the table the
    # autotuner wrote on this GPU model when it ships with the package, else a
    # fresh search (outside the timed region either way)
    tune_file = os.path.join(ROOT, "paper_2308_14490_amd", "tune_mi355x.json")
    if os.path.exists(tune_file) and not args.retune:
        azrbf.tune_load_file(tune_file)
        p0.destroy()
        p0 = problems.plan_for(prob)
        key = next((kk for kk in azrbf.tune_table() if kk.startswith("e")), None)
        tuned = {"engine": True, "source": os.path.relpath(tune_file, ROOT), "key": key}
        if key:
            tuned.update(dict(zip(("C", "L", "chunk"), azrbf.tune_table()[key])))
    else:
        tuned = dict(azrbf.autotune(p0, args.nrhs), source="autotune")
    log("tile shapes:", {kk: tuned.get(kk) for kk in ("source", "key", "C", "L", "chunk", "ms")})
    p0.destroy()
    X = torch.empty((args.nrhs, prob.N), dtype=torch.float64, device=dev)
    rel = torch.empty(args.nrhs, dtype=torch.float64, device=dev)

    def make_plan():
        return azrbf.Plan(1, prob.n, prob.s, prob.T, mask, eps=prob.eps, tau=1e-12, tauZ=1e-12,
                          k=prob.k, refine=1, seed=prob.seed)

    def step(rel_out=None):
        p = make_plan()
        azrbf.solve(p, B, X, rel if rel_out is None else rel_out)
        p.destroy()

    if args.profile_only:
        # per-launch timing on: the library runs its launches one at a time, the
        # mode in which bench's own per-kernel figures are taken
        azrbf.profile_enable(True)
    log(f"workload N={prob.N} M={M} nrhs={args.nrhs} k={k}; warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    # one residual row per timed step, so that every step's solves are gated
    rel_steps = torch.empty((args.steps, args.nrhs), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(rel_steps[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rels = rel_steps.cpu().numpy()
    ms_step = (t1 - t0) * 1e3 / args.steps
    good = int(np.sum(rels <= 1e-10))
    value = good / (t1 - t0)
    log(f"{ms_step:.3f} ms/step, {value:.1f} solves/s, max relres {rels.max():.2e}")
    if args.calibrate:
        a = torch.full((1 << 27,), 1.0, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        b = a * 2.0          # the calibration kernel: reads and writes 2^27 doubles
        torch.cuda.synchronize()
        del a, b
    if args.profile_only:
        azrbf.profile_report()
        azrbf.profile_enable(False)
        return 0

    # per-kernel roofline: the same steps with HIP events around every launch
    azrbf.profile_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    kern = by_kernel(azrbf.profile_report())
    azrbf.profile_enable(False)
    kern.sort(key=lambda r: -r["ms"])
    total_ms = sum(r["ms"] for r in kern)
    dom = kern[0]
    roofline = roofline_of(dom, total_ms)
    fft = [r for r in kern if r["name"].startswith(("col_", "row_", "fused_"))]
    fft_ms = sum(r["ms"] for r in fft)
    fft_passes = {"kernels": len(fft), "share_of_gpu_time": round(fft_ms / total_ms, 3),
                  "achieved": round(sum(r["bytes"] for r in fft) / (fft_ms * 1e-3) / 1e9, 1) if fft_ms else None,
                  "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    if fft_passes["achieved"]:
        fft_passes["frac"] = round(fft_passes["achieved"] / HBM_PEAK_GBS, 4)
    table = [{"name": r["name"], "calls": r["calls"], "avg_us": round(r["ms"] / r["calls"] * 1e3, 2),
              "GBps": round(r["bytes"] / (r["ms"] * 1e-3) / 1e9, 1) if r["ms"] > 0 else None,
              "share": round(r["ms"] / total_ms, 3)} for r in kern[:12]]
    log("dominant kernel", json.dumps(roofline))

    # plain modes
    # every mode counts only right-hand sides whose residual is <= 1e-10
    Bp = B[: args.plain].contiguous()
    Xp = torch.empty((1, prob.N), dtype=torch.float64, device=dev)
    rp = torch.empty((args.plain, 1), dtype=torch.float64, device=dev)
    p = make_plan()                      # warm-up: first launches of the one-vector kernels
    azrbf.solve(p, Bp[0:1], Xp, rp[0])
    p.destroy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.plain):
        p = make_plan()
        azrbf.solve(p, Bp[i:i + 1], Xp, rp[i])
        p.destroy()
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t0
    good_plain = int((rp <= 1e-10).sum())
    plain_problem = good_plain / dt_plain
    log(f"plain per-problem: {good_plain}/{args.plain} at relres <= 1e-10 in {dt_plain * 1e3:.2f} ms")
    p = make_plan()
    azrbf.factor(p)
    azrbf.solve(p, Bp[0:1], Xp, rp[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.plain):
        azrbf.solve(p, Bp[i:i + 1], Xp, rp[i])
    torch.cuda.synchronize()
    plain_resident = int((rp <= 1e-10).sum()) / (time.perf_counter() - t0)
    rb = torch.empty((3, args.nrhs), dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    for i in range(3):
        azrbf.solve(p, B, X, rb[i])
    torch.cuda.synchronize()
    batched_resident = int((rb <= 1e-10).sum()) / (time.perf_counter() - t0)
    p.destroy()
    log(f"plain per-problem {plain_problem:.1f}/s, plain resident {plain_resident:.1f}/s, "
        f"batched resident {batched_resident:.1f}/s")

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"1D batched AZ: N={prob.N} Gaussian RBF centres on [-1,1), eps*h={prob.eh}, "
                               f"s={prob.s}, domain [-0.5,0.5] (M={M}), {args.nrhs} random-trig RHS, "
                               f"k={k}, one refinement pass; step = plan + factor + solve",
                   "N": prob.N, "M": M, "nrhs": args.nrhs, "k": k, "eh": prob.eh},
        "max_relres": float(rels.max()),
        "modes": {"batched_per_problem": round(value, 2), "plain_per_problem": round(plain_problem, 2),
                  "plain_resident_factor": round(plain_resident, 2),
                  "batched_resident_factor": round(batched_resident, 2)},
        "roofline": roofline,
        "fft_passes": fft_passes,
        "tile_shapes": {kk: tuned.get(kk) for kk in ("source", "key", "nvec", "C", "L", "chunk", "ms")},
        "kernels": table,
    }
    if not args.no_served:
        out["served_stream"] = served_vs_plain(args.serve_count, 2024, sides, log)
    out["fft_passes_beyond_cache"] = beyond_cache(log)
    out["copies_1d_n256"] = copies_1d(log)
    out["uneven_1d"] = uneven_1d(log)
    out["million_1d"] = million_1d(log)
    out["million_1d_exact"] = million_1d(log, n=10 ** 6)
    out["transform_paths"] = transform_paths(log)
    if not args.no_2d:
        out["wide_2d"] = wide_2d(log)
        out["poisson_2d_n256"] = bvp_2d(log)
        out["flower_paper_size"] = flower_paper_size(log)
    if not args.no_cpu_baseline:
        log(f"cpu baseline (oracle) at N={args.cpu_n}")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.nrhs)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
