"""Benchmark: S-entries factored per second for Theta-on-S + ICHOL(0) + solves on one MI355X.

Workload (default): 10^6 points on a jittered 1000x1000 grid over [0,1]^2,
Matern nu=1/2 with lengthscale 0.1, rho = 4, maximin ordering, max-rule pattern,
8 N(0,1) right-hand sides.  One step = Theta on S fused into ICHOL(0) (one
launch per DAG level) + the forward and backward triangular solves for all
right-hand sides.  Points, pattern and right-hand sides are resident in HBM
before timing starts; the host analysis (ordering, pattern, schedule), the
upload of the pattern and the device-side symbolic step (the match masks, built
once per pattern) are timed separately and reported beside the result, with the
factorization time without the masks.  Beside the FP64 headline: the mixed
form, its error against the FP64 factor, time to a 1e-10 CG residual for both,
and a bounded serving run (p50/p99 latency).

Prints one JSON line.  value = nnz(S) * steps / timed seconds.
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

METRIC = "S-entries factored/s at N=1e6,d=2 (mixed vs FP64); serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0
PROFILE_JSON = os.path.join(ROOT, "profiles", "ichol_level_jittergrid2d-n1000000-rho4.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1706_02205_amd", "csrc", f) for f in ("kchol.hip", "crmath.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(prec, workload):
    """HBM bytes per launch of the factorization kernel from the committed rocprofv3 counters
    (FETCH_SIZE and WRITE_SIZE, each scaled by its reading for a plain copy of known size),
    or None when the counters were taken on different kernel sources or another workload."""
    try:
        with open(PROFILE_JSON) as f:
            prof = json.load(f)
    except OSError:
        return None
    if prof.get("kernel_source_sha256") != kernel_source_hash() or prof.get("workload") != workload:
        return None
    e = prof.get(prec)
    if not e:
        return None
    return e["fetch_kib_per_launch"] * 1024 * prof["fetch_scale"] + e["write_kib_per_launch"] * 1024 * prof["write_scale"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_copy_gbs(gib=2):
    """Device-to-device copy rate (bytes read + written per second) of a plain gib-GiB copy, GB/s:
    the HBM rate this device delivers to a streaming kernel, reported beside the 8 TB/s spec."""
    import torch
    src = torch.ones(gib * 2 ** 30 // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    t = a.elapsed_time(b) / 5 / 1e3
    rate = 2 * src.numel() * 8 / t / 1e9
    del src, dst
    return rate


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def algorithmic_bytes(prec, nnz, updates):
    """Bytes one factorization must move: per entry a row index read and an L write,
    per Schur update a gathered L value plus its column index (FP64: 12 + 12; MIXED: 8 + 8)."""
    if prec == "fp64":
        return 12 * nnz + 12 * updates
    return 8 * nnz + 8 * updates


def run_gpu(w, prec, steps, warmup, plan, pivot, tau, pcg_tol, keep_L=False, matches=True):
    import torch
    import paper_1706_02205_amd as K
    torch.cuda.synchronize()
    t = time.perf_counter()
    f = K.Factor(plan, prec)
    torch.cuda.synchronize()
    t_upload = time.perf_counter() - t
    xd = torch.from_numpy(w.points).to("cuda")
    bd = torch.from_numpy(w.rhs()).to("cuda")
    out = torch.empty_like(bd)
    # one untimed pass that counts the Schur updates (the algorithmic work)
    f.factorize(xd, w.nu, w.lengthscale, pivot, tau, count_updates=True)
    st = f.stats()
    # the factorization merging row indices, for reference, then the match masks (symbolic, once per
    # pattern, like the host analysis): every timed factorization below uses them
    t_index = None
    match = None
    if matches:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(3):
            f.factorize(xd, w.nu, w.lengthscale, pivot, tau)
        b.record()
        torch.cuda.synchronize()
        t_index = a.elapsed_time(b) / 3 / 1e3
        t = time.perf_counter()
        nbytes = f.build_matches()
        torch.cuda.synchronize()
        match = {"build_s": time.perf_counter() - t, "bytes": nbytes}
    for _ in range(warmup):
        f.factorize(xd, w.nu, w.lengthscale, pivot, tau)
        f.solve(bd, out=out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b, c in ev:
        a.record()
        f.factorize(xd, w.nu, w.lengthscale, pivot, tau)
        b.record()
        f.solve(bd, out=out)
        c.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_fac = np.array([a.elapsed_time(b) for a, b, _ in ev]) / 1e3
    t_sol = np.array([b.elapsed_time(c) for _, b, c in ev]) / 1e3
    st2 = f.stats()
    # the same step through the fused call (forward sweep overlapped with the factorization)
    f.factorize_solve(xd, bd, w.nu, w.lengthscale, pivot, tau, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f.factorize_solve(xd, bd, w.nu, w.lengthscale, pivot, tau, out=out)
    torch.cuda.synchronize()
    wall_fused = time.perf_counter() - t0
    refine = None
    if pcg_tol > 0:
        # time to a pcg_tol residual: factorization + CG on the dense Theta preconditioned by it
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        f.factorize(xd, w.nu, w.lengthscale, pivot, tau)
        sol, info = f.pcg(xd, bd, w.nu, w.lengthscale, tol=pcg_tol, maxit=200)
        b.record()
        torch.cuda.synchronize()
        n2 = float(w.n) ** 2
        refine = {"tol": pcg_tol, "seconds_to_tol": a.elapsed_time(b) / 1e3, "iterations": info.iterations,
                  "converged": info.converged, "max_rel_residual": info.max_rel_residual,
                  "true_rel_residual": info.true_rel_residual, "restarts": info.restarts,
                  "dense_matvec_s": info.t_matvec_ms / 1e3, "precond_s": info.t_precond_ms / 1e3,
                  # products: one per iteration plus the true-residual checks (one per restart, one at the end)
                  "dense_pairs_per_s": n2 * (info.iterations + info.restarts + 1) / (info.t_matvec_ms / 1e3)}
    return dict(wall=wall, wall_fused=wall_fused, t_factor=t_fac, t_solve=t_sol, updates=st.updates, rank=st2.rank,
                nonpositive=st2.nonpositive, shifted=st2.shifted, exp_hard=st2.exp_hard, nonfinite=st2.nonfinite,
                match_errors=st2.match_errors, t_upload=t_upload, t_index=t_index, match=match,
                workspace_bytes=f.workspace_bytes, refine=refine, L=f.export_L() if keep_L else None,
                schedule=dict(zip(("waves_per_block", "persist_max", "unit_order"), f.schedule())))


def cpu_baseline(m):
    """The oracle (brute force, single-threaded ICHOL(0)) on the same workload shape at m*m points."""
    import oracle as O
    from paper_1706_02205_amd import workloads as W
    w = W.large_grid_2d(m)
    P = O.pattern(w.points, w.rho)
    t = time.perf_counter()
    th = O.theta_on_pattern(P, w.nu, w.lengthscale)
    t_theta = time.perf_counter() - t
    t = time.perf_counter()
    O.ichol(P, th)
    t_ichol = time.perf_counter() - t
    return {"value": P.nnz / (t_theta + t_ichol), "unit": "S-entries/s", "cores": O.num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"same recipe at N={m * m} ({m}x{m} jittered grid, Matern nu=1/2 l=0.1, rho=4, nnz={P.nnz}); "
                      f"Theta on S {t_theta:.2f} s on {O.num_threads()} threads + ICHOL(0) {t_ichol:.2f} s on 1 thread"}


def run_batched(args):
    """512 independent instances (N log-uniform in [500, 5e4], Matern-3/2, l ~ U(0.05, 0.3), rho=3, one RHS
    each) factored and solved together: one HIP-graph replay per step, mixed precision."""
    import torch
    import paper_1706_02205_amd as K
    from paper_1706_02205_amd import workloads as W
    inst = W.batched_instances(args.instances)
    xs = [b.points for b in inst]
    t = time.perf_counter()
    plan = K.analyze_batched(xs, 3.0, "max", args.threads)
    t_analysis = time.perf_counter() - t
    info = plan.info()
    log(f"[bench] batched: {len(xs)} instances, N={info['n']}, nnz={info['nnz']}, levels={info['nlevels']}, "
        f"analysis {t_analysis:.1f} s")
    f = K.Factor(plan, args.prec if args.prec != "both" else "mixed")
    pivot, tau = ("zero", 0.0) if f.prec == "fp64" else ("shift", 1e-6)
    xd = torch.from_numpy(np.concatenate(xs)).cuda()
    ed = torch.tensor([b.lengthscale for b in inst], dtype=torch.float64, device="cuda")
    bd = torch.from_numpy(np.concatenate([W.gaussian_rhs(len(b.points), 1, b.rhs_seed) for b in inst])).cuda()
    f.factorize_batched(xd, 1.5, ed, pivot, tau, count_updates=True)
    st = f.stats()
    wpb = f.tune(xd, 1.5, ell_dev=ed, pivot=pivot, tau=tau, reps=2)
    wpb, pm, order = f.schedule()
    log(f"[bench] tuner: {wpb} wavefronts per workgroup, levels with <= {pm} units in persistent launches, "
        f"unit order {order}")

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    # eager factorize + solve with the tuned schedule (persistent launches included)
    eager_s = timed(lambda: (f.factorize_batched(xd, 1.5, ed, pivot, tau), f.solve(bd)))
    # the same step replayed from a HIP graph (one launch per level)
    g = f.capture(xd, bd, 1.5, ell_dev=ed, pivot=pivot, tau=tau)
    graph_s = timed(g.launch)
    ginfo = g.info()
    # and through the fused call (forward sweep overlapped with the factorization)
    out = torch.empty_like(bd)
    fused_s = timed(lambda: f.factorize_solve(xd, bd, 1.5, pivot=pivot, tau=tau, out=out, ell_dev=ed))
    step_s = min(eager_s, graph_s, fused_s)
    log(f"[bench] batched step: eager {eager_s * 1e3:.1f} ms, graph {graph_s * 1e3:.1f} ms ({ginfo['nodes']} nodes), "
        f"fused {fused_s * 1e3:.1f} ms")
    nnz = info["nnz"]
    print(json.dumps({
        "metric": "S-entries factored/s over a batch of independent problems", "value": nnz / step_s,
        "unit": "S-entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-updates/f64-pivots" if f.prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"batched-{len(xs)}-matern32", "instances": len(xs), "n_total": info["n"],
                   "nnz": nnz, "levels": info["nlevels"], "nrhs": 1, "rho": 3.0, "tuned_waves_per_block": wpb,
                   "tuned_persist_max": pm, "tuned_unit_order": order,
                   "step_form": ["eager", "graph", "fused"][int(np.argmin([eager_s, graph_s, fused_s]))]},
        "eager_ms": eager_s * 1e3, "graph_ms": graph_s * 1e3, "fused_ms": fused_s * 1e3, "graph_nodes": ginfo["nodes"],
        "updates": st.updates, "host_analysis_s": t_analysis}), flush=True)


def run_serving(args):
    """Poisson arrivals of factor+solve requests: N log-uniform in [1e3, 2e5], points of intrinsic
    dimension 2 in R^20, Matern-3/2 l=0.2, rho=3, 4 right-hand sides, mixed precision, factors kept
    resident within a 64 GB nnz(S)-proportional budget.  The capacity is measured first (every request
    arriving at once); the same requests are then replayed at 0.5, 0.8 and 1.0 times that rate.  The
    value is p50 latency at 0.8 x capacity; p50/p99 and throughput are reported for every rate."""
    cap, runs = serve_run(args.requests, args.analysis_threads, (0.5, 0.8, 1.0))
    log(f"[bench] serving capacity (all {args.requests} requests at once): {cap:.2f} requests/s")
    for sm in runs:
        log(f"[bench] serving at {sm['load']:.1f} x capacity ({sm['rate_per_s']:.2f}/s): p50 {sm['p50_ms']:.1f} ms, "
            f"p99 {sm['p99_ms']:.1f} ms, {sm['throughput_req_s']:.2f} requests/s")
    head = runs[1]
    print(json.dumps({
        "metric": "serve p50/p99 ms", "value": head["p50_ms"], "unit": "ms", "n_gpus": 1, "steps": args.requests,
        "warmup": 0, "ms_per_step": head["mean_ms"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-updates/f64-pivots", "data": "synthetic",
        "config": {"workload": f"serve-sincos20d-{args.requests}req-load0.8", "rate_per_s": head["rate_per_s"],
                   "capacity_req_s": cap, "n_range": [1000, 200000], "nrhs": 4, "budget_bytes": 64e9},
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "throughput_req_s": head["throughput_req_s"],
        "s_entries_per_s": head["s_entries_per_s"], "peak_inflight": head["peak_inflight"],
        "peak_resident_bytes": head["peak_resident_bytes"],
        "loads": [{k: r[k] for k in ("load", "rate_per_s", "p50_ms", "p99_ms", "throughput_req_s", "peak_inflight")}
                  for r in runs]}), flush=True)


def factor_error_report(plan, points, L64, Lmx, nu, ell, npairs=200_000, seed=1007):
    """The mixed factor against the FP64 factor at full size (the FP64 factor is the oracle's bit for bit
    wherever the oracle can run, see tests/test_gpu_fullpath_250k.py): per column max_k |dL_kj| / max_k |L_kj|
    and ||dL||_F / ||L||_F, plus the sampled error E of Section 4.4 for both factors over the same pairs."""
    import scipy.sparse as sp
    from paper_1706_02205_amd import workloads as W
    perm, _, colptr, rowidx = plan.export()
    n, nnz = len(perm), int(colptr[-1])
    dL = np.abs(Lmx - L64)
    col_err = np.maximum.reduceat(dL, colptr[:-1])
    col_max = np.maximum.reduceat(np.abs(L64), colptr[:-1])
    per_col = col_err / np.where(col_max > 0, col_max, 1.0)
    frob = float(np.linalg.norm(Lmx - L64) / np.linalg.norm(L64))
    del dL
    # rows of L (CSR) for (LL^T)_ab = row a . row b; the CSC -> CSR permutation once for both factors
    idx = sp.csc_matrix((np.arange(nnz, dtype=np.float64), rowidx, colptr), shape=(n, n)).tocsr()
    order = idx.data.astype(np.int64)
    xh = points[perm]
    pairs = W.random_pairs(n, npairs, seed)
    out = {"per_column_max_rel": float(per_col.max()), "per_column_median_rel": float(np.median(per_col)),
           "frobenius_rel": frob, "sampled_pairs": npairs}
    for name, L in (("fp64", L64), ("mixed", Lmx)):
        Lr = sp.csr_matrix((L[order], idx.indices, idx.indptr), shape=(n, n))
        num = den = 0.0
        for c in range(0, npairs, 20000):
            a, b = pairs[c:c + 20000, 0], pairs[c:c + 20000, 1]
            llt = np.asarray(Lr[a].multiply(Lr[b]).sum(axis=1)).ravel()
            r = np.sqrt(((xh[a] - xh[b]) ** 2).sum(axis=1)) / ell
            if nu == 0.5:
                th = np.exp(-r)
            elif nu == 1.5:
                th = (1 + np.sqrt(3) * r) * np.exp(-np.sqrt(3) * r)
            else:
                th = (1 + np.sqrt(5) * r + 5 * r * r / 3) * np.exp(-np.sqrt(5) * r)
            num += float(((llt - th) ** 2).sum())
            den += float((th ** 2).sum())
        out[f"sampled_E_{name}"] = float(np.sqrt(num / den))
    return out


def serve_run(requests, analysis_threads, loads=(0.8,)):
    """Poisson arrivals of factor+solve requests (N log-uniform in [1e3, 2e5], points of intrinsic
    dimension 2 in R^20, Matern-3/2 l=0.2, rho=3, 4 right-hand sides, mixed precision, 64 GB of resident
    factors at most).  Capacity first (every request arriving at once), then the same requests at each
    load fraction of it; p50/p99 latency (arrival -> solution on the host) and throughput."""
    from paper_1706_02205_amd import serve
    from paper_1706_02205_amd import workloads as W
    reqs = W.serving_trace(requests, 1.0)  # arrivals for rate 1/s; scaled below
    pts = [r.points for r in reqs]
    rhs = [W.gaussian_rhs(len(r.points), 4, r.rhs_seed) for r in reqs]

    def serve_at(rate):
        scale = 0.0 if rate is None else 1.0 / rate
        trace = [(r.arrival_s * scale, p, b) for r, p, b in zip(reqs, pts, rhs)]
        srv = serve.Server(1.5, 0.2, 3.0, prec="mixed", budget_bytes=64e9, max_inflight=16, nstreams=4,
                           analysis_threads=analysis_threads)
        st = srv.run(trace)
        srv.close()
        return st.summary()

    cap = serve_at(None)["throughput_req_s"]
    runs = []
    for frac in loads:
        sm = serve_at(frac * cap)
        sm["rate_per_s"] = frac * cap
        sm["load"] = frac
        runs.append(sm)
    return cap, runs


def sampled_errors(plan, points, factors, nu, ell, npairs, seed):
    """Sampled error E of Section 4.4 for each factor (dict name -> L in CSC order) over the same pairs."""
    import scipy.sparse as sp
    from paper_1706_02205_amd import workloads as W
    perm, _, colptr, rowidx = plan.export()
    n, nnz = len(perm), int(colptr[-1])
    idx = sp.csc_matrix((np.arange(nnz, dtype=np.float64), rowidx, colptr), shape=(n, n)).tocsr()
    order = idx.data.astype(np.int64)
    xh = points[perm]
    pairs = W.random_pairs(n, npairs, seed)
    out = {}
    for name, L in factors.items():
        Lr = sp.csr_matrix((L[order], idx.indices, idx.indptr), shape=(n, n))
        num = den = 0.0
        for c in range(0, npairs, 20000):
            a, b = pairs[c:c + 20000, 0], pairs[c:c + 20000, 1]
            llt = np.asarray(Lr[a].multiply(Lr[b]).sum(axis=1)).ravel()
            r = np.sqrt(((xh[a] - xh[b]) ** 2).sum(axis=1)) / ell
            if nu == 0.5:
                th = np.exp(-r)
            elif nu == 1.5:
                th = (1 + np.sqrt(3) * r) * np.exp(-np.sqrt(3) * r)
            else:
                th = (1 + np.sqrt(5) * r + 5 * r * r / 3) * np.exp(-np.sqrt(5) * r)
            num += float(((llt - th) ** 2).sum())
            den += float((th ** 2).sum())
        out[name] = float(np.sqrt(num / den))
    return out


def run_supernodal(args):
    """N = 2e5 points iid uniform in [0,1]^3, l=0.2, rho=3 (Matern-5/2 by default, --nu 0.5 for the paper's own
    3-D kernel): supernodal ordering and block-closed pattern, mixed factorization with SHIFT (tau = 1e-6) by
    supernodal groups on the matrix cores (the step), beside the entry-wise factorization of the same plan
    (with match masks when they fit in memory); counts and the sampled error E of both."""
    import torch
    import paper_1706_02205_amd as K
    from paper_1706_02205_amd import workloads as W
    w = W.uniform_3d()
    nu = args.nu if args.nu > 0 else w.nu
    rho = args.rho if args.rho > 0 else w.rho
    t = time.perf_counter()
    plan = K.analyze_supernodal(w.points, rho, args.threads)
    t_analysis = time.perf_counter() - t
    info = plan.info()
    sptr = plan.supernodes()
    sizes = np.diff(sptr)
    log(f"[bench] supernodal 3-D: N={w.n} nu={nu} rho={rho} nnz={info['nnz']} supernodes={len(sizes)} "
        f"(points in supernodes >= 16: {sizes[sizes >= 16].sum() / w.n:.2f}) analysis {t_analysis:.1f} s")
    xd = torch.from_numpy(w.points).cuda()
    f = K.Factor(plan, "mixed")
    pivot, tau = "shift", 1e-6

    def timed(reps):
        f.factorize(xd, nu, w.lengthscale, pivot, tau)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            f.factorize(xd, nu, w.lengthscale, pivot, tau)
        torch.cuda.synchronize()
        st = f.stats()
        return (time.perf_counter() - t0) / reps, {"shifted": st.shifted, "nonfinite": st.nonfinite}

    t_groups, c_groups = timed(args.steps)
    L_groups = f.export_L()
    f.use_groups(False)
    t_entry, c_entry = timed(max(1, args.steps // 3))
    L_entry = f.export_L()
    t_masks = None
    if f.match_bytes() < 100e9:
        f.build_matches()
        t_masks, _ = timed(max(1, args.steps // 3))
        f.drop_matches()
    log(f"[bench] mixed factorization: groups on MFMA {t_groups * 1e3:.1f} ms, entry-wise {t_entry * 1e3:.1f} ms"
        + (f", entry-wise with match masks {t_masks * 1e3:.1f} ms" if t_masks else "")
        + f"; shifted {c_groups['shifted']}, non-finite {c_groups['nonfinite']} (groups) / {c_entry['nonfinite']} (entry-wise)")
    f.use_groups(True)
    t = time.perf_counter()
    errs = sampled_errors(plan, w.points, {"groups": L_groups, "entrywise": L_entry}, nu, w.lengthscale, 200_000, 1005)
    log(f"[bench] sampled error E (200,000 pairs): groups {errs['groups']:.3e}, entry-wise {errs['entrywise']:.3e} "
        f"({time.perf_counter() - t:.1f} s)")
    nnz = info["nnz"]
    name = f"uniform3d-n{w.n}-matern{int(round(2 * nu))}2-rho{rho:g}-supernodal"
    print(json.dumps({
        "metric": "S-entries factored/s (supernodal pattern, 3-D, mixed)", "value": nnz / t_groups,
        "unit": "S-entries/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": t_groups * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-updates/f64-pivots", "data": "synthetic",
        "config": {"workload": name, "n": w.n, "d": 3, "nu": nu, "rho": rho, "supernodes": int(len(sizes)),
                   "max_supernode": int(sizes.max()), "points_in_supernodes_ge16": float(sizes[sizes >= 16].sum() / w.n),
                   "nnz": nnz, "pivot": "shift 1e-6"},
        "groups_ms": t_groups * 1e3, "entrywise_ms": t_entry * 1e3,
        "entrywise_match_masks_ms": t_masks * 1e3 if t_masks else None,
        "counts_groups": c_groups, "counts_entrywise": c_entry,
        "sampled_error_E": errs, "sampled_error_pairs": 200_000,
        "host_analysis_s": t_analysis}), flush=True)


def run_dense(args):
    """The dense Theta product alone (conjugate gradients' matrix product): Y = Theta X on the 10^6-point
    grid with 8 right-hand sides, Theta generated on the fly (10^12 kernel evaluations per product)."""
    import torch
    import paper_1706_02205_amd as K
    from paper_1706_02205_amd import workloads as W
    w = W.large_grid_2d()
    x = torch.from_numpy(w.points).cuda()
    X = torch.from_numpy(w.rhs()).cuda()
    for _ in range(args.warmup):
        K.dense_matvec(x, X, w.nu, w.lengthscale)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        K.dense_matvec(x, X, w.nu, w.lengthscale)
    b.record()
    torch.cuda.synchronize()
    t = a.elapsed_time(b) / 1e3 / args.steps
    pairs = float(w.n) ** 2
    print(json.dumps({
        "metric": "kernel evaluations/s in the dense Theta product", "value": pairs / t, "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"dense-{w.name}", "n": w.n, "nrhs": w.nrhs, "kernel": f"matern nu={w.nu} l={w.lengthscale}"}}),
        flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=1000, help="m for the m x m jittered grid")
    ap.add_argument("--prec", default="both", choices=["fp64", "mixed", "both"],
                    help="both: FP64 is the headline value, the mixed form is reported beside it")
    ap.add_argument("--cpu-grid", type=int, default=250, help="m of the oracle's CPU-baseline sample (0 = skip)")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--pcg-tol", type=float, default=1e-10,
                    help="also time CG on the dense Theta to this residual with each factor (0 = skip)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration for profiles)")
    ap.add_argument("--workload", default="grid", choices=["grid", "batched", "serve", "supernodal3d", "dense"],
                    help="grid: the 10^6-point benchmark (default); batched: 512 independent instances; "
                         "serve: Poisson trace of factor+solve requests; dense: the dense Theta product alone")
    ap.add_argument("--requests", type=int, default=120)
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="grid workload: also serve this many requests at 0.8 x measured capacity (0 = skip)")
    ap.add_argument("--error-pairs", type=int, default=200_000,
                    help="grid workload: sampled pairs for the mixed-vs-FP64 error report (0 = skip)")
    ap.add_argument("--nu", type=float, default=0.0, help="supernodal3d: Matern smoothness (default: the workload's)")
    ap.add_argument("--rho", type=float, default=0.0, help="supernodal3d: rho (default: the workload's)")
    ap.add_argument("--no-matches", action="store_true",
                    help="factor without match masks (index merge), e.g. to compare")
    ap.add_argument("--analysis-threads", type=int, default=12)
    ap.add_argument("--instances", type=int, default=512)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the factorization is a single-device kernel sequence).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "serve":
        run_serving(args)
        return
    if args.workload == "supernodal3d":
        run_supernodal(args)
        return
    if args.workload == "dense":
        run_dense(args)
        return

    import paper_1706_02205_amd as K
    from paper_1706_02205_amd import workloads as W

    w = W.large_grid_2d(args.grid)
    log(f"[bench] workload {w.name}: {w.description}")
    t = time.perf_counter()
    plan = K.analyze(w.points, w.rho, "max", args.threads)
    t_analysis = time.perf_counter() - t
    info = plan.info()
    log(f"[bench] host analysis {t_analysis:.2f} s: nnz={info['nnz']} levels={info['nlevels']} "
        f"units={info['nunits']}")

    if args.copy_mib > 0:
        import torch
        src = torch.ones(args.copy_mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 x {args.copy_mib} MiB device-to-device")
        del src, dst

    copy_gbs = measured_copy_gbs()
    log(f"[bench] device-to-device copy: {copy_gbs:.0f} GB/s (read + write)")
    precs = ["fp64", "mixed"] if args.prec == "both" else [args.prec]
    nnz = info["nnz"]
    entries = {}
    factors = {}
    for prec in precs:
        pivot, tau = ("zero", 0.0) if prec == "fp64" else ("shift", 1e-6)
        r = run_gpu(w, prec, args.steps, args.warmup, plan, pivot, tau, args.pcg_tol,
                    keep_L=args.error_pairs > 0 and len(precs) == 2, matches=not args.no_matches)
        factors[prec] = r.pop("L")
        # a step is factorize + solve: as two calls, or as the fused call that overlaps the forward sweep
        # with the factorization (bitwise the same result); the faster of the two is the step
        step_sep, step_fused = r["wall"] / args.steps, r["wall_fused"] / args.steps
        step_s = min(step_sep, step_fused)
        log(f"[bench] {prec}: step {step_sep * 1e3:.2f} ms as two calls, {step_fused * 1e3:.2f} ms fused")
        tf = float(np.mean(r["t_factor"]))
        ts = float(np.mean(r["t_solve"]))
        log(f"[bench] {prec}: factor {tf * 1e3:.2f} ms  solve {ts * 1e3:.2f} ms  updates={r['updates']}")
        if r["match"]:
            log(f"[bench] {prec}: match masks {r['match']['bytes'] / 1e9:.1f} GB built in {r['match']['build_s']:.2f} s; "
                f"factor without them {r['t_index'] * 1e3:.2f} ms")
        B = algorithmic_bytes(prec, nnz, r["updates"])
        launches = info["nlevels"]
        achieved = (B / launches) / (tf / launches) / 1e9
        traffic = measured_traffic(prec, w.name)
        entries[prec] = {
            "value": nnz / step_s, "ms_per_step": step_s * 1e3,
            "step_ms": {"factorize_then_solve": step_sep * 1e3, "factorize_solve_fused": step_fused * 1e3},
            "dtype": "f64" if prec == "fp64" else "f32-updates/f64-pivots", "pivot": pivot,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                         "measured_copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                         "kernel": ("ichol_level (Theta fused, match masks)" if r["match"] else
                                    "ichol_level (Theta fused, index merge)") + ", one launch per DAG level",
                         "launches_per_factorization": launches,
                         "algorithmic_bytes_per_launch": B / launches,
                         "avg_launch_ms": tf / launches * 1e3},
            "factor_only": {"value": nnz / tf, "unit": "S-entries/s", "ms": tf * 1e3},
            "solve_ms": ts * 1e3, "updates": r["updates"], "rank": r["rank"], "nonpositive": r["nonpositive"],
            "shifted": r["shifted"], "exp_hard": r["exp_hard"], "nonfinite": r["nonfinite"],
            "match_errors": r["match_errors"], "upload_s": r["t_upload"],
            "workspace_bytes": r["workspace_bytes"], "schedule": r["schedule"],
            # symbolic match masks: built once per pattern (like the host analysis), not in the timed steps
            "match_masks": r["match"],
            "factor_ms_without_masks": r["t_index"] * 1e3 if r["t_index"] is not None else None,
        }
        if r["refine"] is not None:
            entries[prec]["refine"] = r["refine"]
            log(f"[bench] {prec}: {r['refine']['iterations']} CG iterations to {args.pcg_tol:g} in "
                f"{r['refine']['seconds_to_tol']:.2f} s")
    head = entries[precs[0]]
    result = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "S-entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "kernel": f"matern nu={w.nu} l={w.lengthscale}",
                   "rho": w.rho, "rule": "max", "nrhs": w.nrhs, "prec": precs[0], "pivot": head["pivot"]},
        "roofline": head["roofline"],
        "factor_only": head["factor_only"],
        "step_ms": head["step_ms"],
        "solve_ms": head["solve_ms"],
        "nnz": nnz, "updates": head["updates"], "rank": head["rank"], "nonpositive": head["nonpositive"],
        "shifted": head["shifted"], "exp_hard": head["exp_hard"], "nonfinite": head["nonfinite"],
        "host_analysis_s": t_analysis, "host_analysis_split_s": [info["t_order_s"], info["t_pattern_s"],
                                                                 info["t_schedule_s"]],
        "upload_s": head["upload_s"], "workspace_bytes": head["workspace_bytes"], "schedule": head["schedule"],
    }
    if "refine" in head:
        result["refine"] = head["refine"]
    if "mixed" in entries and precs[0] != "mixed":
        result["mixed"] = entries["mixed"]
        if factors.get("fp64") is not None and factors.get("mixed") is not None:
            t = time.perf_counter()
            rep = factor_error_report(plan, w.points, factors["fp64"], factors["mixed"], w.nu, w.lengthscale,
                                      args.error_pairs)
            log(f"[bench] mixed vs fp64 factor: per-column max rel {rep['per_column_max_rel']:.2e}, Frobenius "
                f"{rep['frobenius_rel']:.2e}; sampled E fp64 {rep['sampled_E_fp64']:.3e} mixed "
                f"{rep['sampled_E_mixed']:.3e} ({time.perf_counter() - t:.1f} s)")
            result["mixed"]["error_vs_fp64"] = rep
    factors.clear()
    if args.serve_requests > 0:
        # the second half of the metric: serving latency, a bounded run at 0.8 x the capacity measured here
        t = time.perf_counter()
        cap, runs = serve_run(args.serve_requests, args.analysis_threads, (0.8,))
        sm = runs[0]
        log(f"[bench] serving {args.serve_requests} requests: capacity {cap:.2f}/s; at 0.8 x: p50 {sm['p50_ms']:.1f} ms "
            f"p99 {sm['p99_ms']:.1f} ms, {sm['throughput_req_s']:.2f} requests/s ({time.perf_counter() - t:.1f} s)")
        result["serve"] = {"workload": f"serve-sincos20d-{args.serve_requests}req", "requests": args.serve_requests,
                           "capacity_req_s": cap, "load": 0.8, "rate_per_s": sm["rate_per_s"],
                           "p50_ms": sm["p50_ms"], "p99_ms": sm["p99_ms"], "throughput_req_s": sm["throughput_req_s"],
                           "peak_inflight": sm["peak_inflight"], "prec": "mixed", "nrhs": 4,
                           "n_range": [1000, 200000]}
    if args.cpu_grid > 0:
        log(f"[bench] CPU baseline: oracle at {args.cpu_grid}x{args.cpu_grid}")
        result["cpu_baseline"] = cpu_baseline(args.cpu_grid)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
