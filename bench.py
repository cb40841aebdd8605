#!/usr/bin/env python3
"""Benchmark: FP64 supernodal Cholesky factor + solve on one MI355X.

One step = one pass of the device hot path over resident inputs: value load,
supernodal factorization (diagonal factorizations, panel solves, update blocks
scattered through relative indices, level schedule) and one forward/backward
solve.  The symbolic analysis runs once before the timed region (it is reused
by every refactorization, as in the paper's factor/solve split) and is
reported separately.

Metric: factorization GFLOP/s with F = sum_j colcount(j)^2 over the exact
structure of L, divided by the device time of one factorization (value load
included), plus p50/p99 latency of repeated single-RHS solves.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Cholesky factor GFLOP/s FP64 vs FP32+IR @1e-10 bwd err; p50/p99 solve latency"
FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBPS = 8000.0
HBM_PEAK_GBS = 8000.0

WORKLOAD_TEXT = {
    "lap3d_7pt_64": "3D 7-point Laplacian 64^3 (n=262144), lognormal(0,1) edge weights, "
                    "diag = row sum + 1e-6, geometric nested dissection, amalgamation 0.1, "
                    "1 RHS N(0,1)",
    "lap2d_5pt_64": "2D 5-point Laplacian 64x64 (n=4096), unit weights + 1e-3 shift, "
                    "geometric nested dissection, 1 RHS N(0,1)",
    "elast27_48": "3D 27-point stencil, 3 unknowns per node, 48^3 grid (n=331776): random "
                  "3x3 SPD (Wishart) edge blocks, diagonal blocks dominant + 1e-3 shift, "
                  "geometric nested dissection, amalgamation 0.1, 8 RHS N(0,1)",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def update_flops(sym) -> float:
    """Flops of the update task over all supernodes: the lower triangle
    (diagonal included) of L21 L21^T, w * r * (r + 1) per supernode."""
    _, _, sn, _ = sym.export()
    rp, _ = sym.rows()
    w = np.diff(sn).astype(np.float64)
    r = np.diff(rp).astype(np.float64) - w
    return float(np.sum(w * r * (r + 1.0)))


def hbm_bytes(sym) -> dict:
    """Algorithmic HBM bytes of the memory-bound phases, FP64:
    - one single-RHS solve: the stored factor read forward and backward plus
      the 4-byte row index of every row below a diagonal block, both ways:
      2 (8 nnz_stored + 4 sum_s r_s);
    - the update scatter of one factorization: a 16-byte read-modify-write of
      the target for every entry of the lower triangle of L21 L21^T:
      16 sum_s r_s (r_s + 1) / 2."""
    _, _, sn, _ = sym.export()
    rp, _ = sym.rows()
    w = np.diff(sn).astype(np.float64)
    r = np.diff(rp).astype(np.float64) - w
    return {"solve": 2.0 * (8.0 * sym.info()["nnz_stored"] + 4.0 * float(r.sum())),
            "scatter": 16.0 * float(np.sum(r * (r + 1.0) / 2.0))}


def backward_error(p, x, b):
    import scipy.sparse as sp

    A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
    A = A + sp.tril(A, -1).T
    r = b - A @ x
    anorm = abs(A).sum(axis=1).max()
    return float(np.abs(r).max() / (anorm * np.abs(x).max() + np.abs(b).max()))


def cpu_baseline(name, sample_dims, repeat=0):
    """The oracle (plain left-looking column Cholesky, one core) timed on a
    bounded sample: the same workload recipe on a smaller grid."""
    saved = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    try:
        os.sched_setaffinity(0, {sorted(saved)[0]})
    except (AttributeError, OSError, TypeError):
        pass
    try:
        return _cpu_baseline_pinned(name, sample_dims, repeat)
    finally:
        if saved is not None:
            os.sched_setaffinity(0, saved)


def _cpu_baseline_pinned(name, sample_dims, repeat):
    import oracle
    from paper_1608_00044_amd import inputs

    p = inputs.make_workload(name, repeat=repeat, nrhs=0, dims=sample_dims)
    Cp, Ci, Cx, _ = oracle.permute(p.n, p.colptr, p.rowind, p.values, p.perm)
    sym = oracle.symbolic(p.n, Cp, Ci)
    t0 = time.perf_counter()
    st, _ = oracle.factor(p.n, Cp, Ci, Cx, sym)
    dt = time.perf_counter() - t0
    if st != 0:
        raise RuntimeError("oracle failed on the sample")
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 1
    return {"value": sym.flops / dt / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": "same recipe on a %s grid (n=%d, F=%.3e), numeric factorization only, "
                      "%.1f s" % ("x".join(map(str, sample_dims)), p.n, sym.flops, dt)}


def _oracle_batch_share(job):
    """Pool worker: the oracle's whole pipeline (permute, symbolic, factor,
    one-RHS solve) on members `ks` of the batch, each timed alone."""
    count, ks = job
    import oracle
    from paper_1608_00044_amd import inputs

    out = []
    for p in inputs.make_batch(count=count, members=ks):
        t0 = time.perf_counter()
        Cp, Ci, Cx, _ = oracle.permute(p.n, p.colptr, p.rowind, p.values, p.perm)
        sym = oracle.symbolic(p.n, Cp, Ci)
        st, Lx = oracle.factor(p.n, Cp, Ci, Cx, sym)
        if st == 0:
            oracle.solve(p.n, sym, Lx, p.perm, p.rhs[:, 0])
        out.append((time.perf_counter() - t0, float(sym.flops), int(st)))
    return out


def cpu_batch_baseline(count, sample, max_workers=16):
    """The oracle on the first `sample` matrices of the batched workload,
    spread over the host's cores by a process pool (members dealt round
    robin): the one-core sum and the pool's makespan (the slowest worker's
    summed compute time), scaled to matrices/s."""
    import multiprocessing

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 1
    workers = max(1, min(cores, max_workers, sample))
    jobs = [(count, list(range(w, sample, workers))) for w in range(workers)]
    t0 = time.perf_counter()
    with multiprocessing.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_batch_share, jobs)
    wall = time.perf_counter() - t0
    if any(st != 0 for r in res for _, _, st in r):
        raise RuntimeError("oracle failed on a batch member")
    per_worker = [sum(t for t, _, _ in r) for r in res]
    one_core = sum(per_worker)
    makespan = max(per_worker)
    flops = sum(f for r in res for _, f, _ in r)
    return {"value": sample / makespan, "unit": "matrices/s", "cores": workers, "kind": "oracle",
            "sample": "first %d of the %d matrices: permute + symbolic + factor + one-RHS "
                      "solve each; %d worker processes, members dealt round robin"
                      % (sample, count, workers),
            "one_core_sum_s": one_core, "makespan_s": makespan, "pool_wall_s": wall,
            "one_core_matrices_per_s": sample / one_core,
            "factor_flops_F": flops}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/), or None when there is none for this workload or the kernel's
    source has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "%s_traffic_%s.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, kv.get("source", ""))
    if "traffic_bytes_per_launch" not in kv or not os.path.isfile(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != kv.get("source_sha256"):
        return None
    return float(kv["traffic_bytes_per_launch"])


def mixed_precision(name, steps, warmup, tol=1e-10):
    """FP64 factor + solve against FP32 factor + FP64 refinement to a normwise
    backward error <= tol, on the same resident workload and right-hand sides."""
    import torch

    from paper_1608_00044_amd import inputs, spchol

    p = inputs.make_workload(name)
    k = p.rhs.shape[1]
    dev = torch.device("cuda:0")
    vals = torch.from_numpy(p.values).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(p.rhs)).to(dev)
    stream = torch.cuda.current_stream()
    out = {"workload": name, "description": WORKLOAD_TEXT.get(name, name), "n": p.n,
           "nrhs": k, "tol": tol}
    for prec in (0, 1):
        sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=150,
                             amalg_ratio=p.meta["amalg"], precision=prec)
        F = sym.info()["flops"]
        num = spchol.factor(sym, vals)
        if num.status() != 0:
            raise RuntimeError("factor status %d (precision %d)" % (num.status(), prec))
        x = None
        for _ in range(max(1, warmup)):
            num.refactor(vals)
            if prec == 0:
                x = num.solve(b, x=x)
            else:
                x, _, _ = num.solve_refine(b, x=x, tol=tol, max_iter=20)
        torch.cuda.synchronize()
        f_ms, s_ms, iters, berr = [], [], [], None
        for _ in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            num.refactor(vals)
            e1.record(stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if prec == 0:
                x = num.solve(b, x=x)
                torch.cuda.synchronize()
            else:
                x, it, berr = num.solve_refine(b, x=x, tol=tol, max_iter=20)
                iters.append(it)
            s_ms.append((time.perf_counter() - t0) * 1e3)
            f_ms.append(e0.elapsed_time(e1))
        xs = x.cpu().numpy()
        eta = max(backward_error(p, xs[:, c], p.rhs[:, c]) for c in range(k))
        fm, sm = float(np.mean(f_ms)), float(np.mean(s_ms))
        key = "fp64" if prec == 0 else "fp32_ir"
        out[key] = {"factor_ms": fm, "factor_gflops": F / (fm * 1e-3) / 1e9,
                    "solve_ms": sm, "total_ms": fm + sm, "backward_error": eta}
        if prec == 1:
            out[key]["refine_iters"] = float(np.mean(iters))
            out[key]["fp64_blocks"] = num.info()["fp64_blocks"]
            out[key]["solve_ms_note"] = "iterative refinement: residuals in FP64, corrections " \
                                        "with the FP32 factor, until every column meets tol"
        log("mixed %s: factor %.2f ms (%.1f GFLOP/s), solve %.2f ms, eta %.2e" %
            (key, fm, F / (fm * 1e-3) / 1e9, sm, eta))
        num.free()
        sym.free()
    out["speedup_fp32_ir_vs_fp64"] = out["fp64"]["total_ms"] / out["fp32_ir"]["total_ms"]
    return out


def batched(count, steps, precision, tol=1e-10, tune_options=True, options=None):
    """Batch of independent 2D Laplacians (BATCH_RECIPE): the analysis options
    tuned on this batch (amalgamation ratio, cap), one batched analysis, then
    timed steps of factorization + one-RHS solve (FP64) or factorization +
    refinement to tol (FP32)."""
    import torch

    from paper_1608_00044_amd import inputs, spchol, tune

    t0 = time.perf_counter()
    probs = inputs.make_batch(count=count)
    gen_s = time.perf_counter() - t0
    vals_h, rhs_h = inputs.stack_batch(probs)
    mats = [(p.n, p.colptr, p.rowind, p.perm) for p in probs]
    vals = torch.from_numpy(vals_h).to("cuda:0")
    b = torch.from_numpy(np.ascontiguousarray(rhs_h)).to("cuda:0")
    opts, table = dict(tune.BASE, **(options or {})), None
    if tune_options:
        t0 = time.perf_counter()
        opts, table = tune.tune_batch(mats, vals, b, precision)
        log("batch tuning (%.1f s): %s" % (time.perf_counter() - t0, opts))
    t0 = time.perf_counter()
    sym = spchol.analyze_batch(mats, precision=precision, **opts)
    an_ms = (time.perf_counter() - t0) * 1e3
    inf = sym.info()
    num = spchol.factor(sym, vals)
    if num.status() != 0:
        raise RuntimeError("batched factor status %d" % num.status())
    x = None
    stream = torch.cuda.current_stream()
    f_ms, s_ms, iters = [], [], []
    for k in range(steps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        num.refactor(vals)
        e1.record(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if precision == 0:
            x = num.solve(b, x=x)
            torch.cuda.synchronize()
        else:
            x, it, berr = num.solve_refine(b, x=x, tol=tol, max_iter=20)
            iters.append(it)
        if k > 0:  # the first step captures the solve graphs
            s_ms.append((time.perf_counter() - t0) * 1e3)
            f_ms.append(e0.elapsed_time(e1))
    xs = x.cpu().numpy().ravel()
    worst, off = 0.0, 0
    for p in probs[:50]:
        worst = max(worst, backward_error(p, xs[off:off + p.n], p.rhs[:, 0]))
        off += p.n
    fm, sm = float(np.mean(f_ms)), float(np.mean(s_ms))
    out = {"count": count, "n_total": inf["n"], "nnz_L": inf["nnz_l"], "flops_F": inf["flops"],
           "nsup": inf["nsup"], "levels": inf["nlevels"], "precision": ["fp64", "fp32_ir"][precision],
           "generate_s": gen_s, "analyze_ms": an_ms, "factor_ms": fm,
           "factor_gflops": inf["flops"] / (fm * 1e-3) / 1e9, "solve_ms": sm,
           "matrices_per_s": count / ((fm + sm) * 1e-3),
           "backward_error_first50": worst,
           "launches": "level-set launches over all matrices at once",
           "options": opts}
    if table is not None:
        out["tuning"] = [dict(t["options"], stage=t["stage"], ms=t["ms"], nsup=t["nsup"],
                              levels=t["levels"]) for t in table]
    if precision == 1:
        out["refine_iters"] = float(np.mean(iters))
    log("batch %s: factor %.2f ms (%.1f GFLOP/s), solve %.2f ms, %.0f matrices/s" %
        (out["precision"], fm, out["factor_gflops"], sm, out["matrices_per_s"]))
    num.free()
    sym.free()
    return out


SERVE_RECIPE = dict(rate=200.0, patterns_2d=16, patterns_3d=16, side2d=(32, 256),
                    side3d=(16, 48), sigma=1.0, solve_only=0.3, nrhs=(1, 4, 16, 64),
                    value_sets=2)


def serving(requests, seed=5000):
    """Poisson request stream over 32 resident patterns through the request
    server; reports latency percentiles and throughput."""
    import torch

    from paper_1608_00044_amd import inputs, spchol

    r = SERVE_RECIPE
    rng = np.random.Generator(np.random.PCG64(seed))
    sides2 = np.linspace(r["side2d"][0], r["side2d"][1], r["patterns_2d"]).round().astype(int)
    sides3 = np.linspace(r["side3d"][0], r["side3d"][1], r["patterns_3d"]).round().astype(int)
    dims = [(int(s), int(s)) for s in sides2] + [(int(s),) * 3 for s in sides3]
    probs, vals = [], []
    for k, d in enumerate(dims):
        sets = [inputs.make_grid_problem("lap", d, seed + 100 * k + v, sigma=r["sigma"],
                                         shift=1e-3, nrhs=0) for v in range(r["value_sets"])]
        probs.append(sets[0])
        vals.append([torch.from_numpy(p.values).to("cuda:0") for p in sets])
    torch.zeros(1, device="cuda:0")
    srv = spchol.Server(max_inflight=16, max_nrhs=max(r["nrhs"]))
    syms = [spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=150, amalg_ratio=0.1)
            for p in probs]
    pids = [srv.add_pattern(s) for s in syms]
    # requests: pattern, kind, nrhs, arrival time
    gaps = rng.exponential(1.0 / r["rate"], size=requests)
    arrive = np.cumsum(gaps)
    pat = rng.integers(len(probs), size=requests)
    kind = (rng.random(requests) < r["solve_only"]).astype(int)
    nrhs = rng.choice(r["nrhs"], size=requests)
    # every pattern's first request factors
    seen = set()
    for i in range(requests):
        if pat[i] not in seen:
            kind[i] = 0
            seen.add(pat[i])
    bufs = {}
    for k in range(len(probs)):
        n = probs[k].n
        bufs[k] = (torch.randn((max(r["nrhs"]), n), dtype=torch.float64, device="cuda:0").t(),)
    xs = [torch.empty((int(nrhs[i]), probs[pat[i]].n), dtype=torch.float64,
                      device="cuda:0").t() for i in range(requests)]
    torch.cuda.synchronize()
    tickets = []
    t0 = time.perf_counter()
    for i in range(requests):
        wait = t0 + arrive[i] - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        k = int(pat[i])
        b = bufs[k][0][:, : int(nrhs[i])]
        v = vals[k][i % r["value_sets"]] if kind[i] == 0 else None
        tickets.append(srv.submit(pids[k], b, xs[i], values=v))
    res = [srv.wait(t) for t in tickets]
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.destroy()
    lat = np.array([q["latency_ms"] for q in res])
    ok = sum(1 for q in res if q["status"] == 0)
    cols = int(sum(int(nrhs[i]) for i in range(requests) if res[i]["status"] == 0))
    out = {"requests": requests, "rate_per_s": r["rate"], "patterns": len(probs),
           "ok": ok, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "requests_per_s": requests / wall,
           "solves_per_s": cols / wall, "peak_inflight": st["peak_inflight"],
           "peak_bytes": st["peak_bytes"], "evictions": st["evictions"],
           "recipe": "Poisson arrivals at %g/s over %d 2D (side %d..%d) and %d 3D 7-point "
                     "(side %d..%d) patterns, lognormal(0,%g) weights, %d%% solve-only on the "
                     "current factor, nrhs uniform in %s" % (
                         r["rate"], r["patterns_2d"], r["side2d"][0], r["side2d"][1],
                         r["patterns_3d"], r["side3d"][0], r["side3d"][1], r["sigma"],
                         int(100 * r["solve_only"]), list(r["nrhs"]))}
    log("serve: p50 %.2f ms p99 %.2f ms, %.1f req/s, %.0f solves/s, peak inflight %d" %
        (out["p50_ms"], out["p99_ms"], out["requests_per_s"], out["solves_per_s"],
         out["peak_inflight"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lap3d_7pt_64")
    ap.add_argument("--solves", type=int, default=200)
    ap.add_argument("--sched", type=int, default=0, choices=(0, 1, 2),
                    help="0 level sets, 1 with lookahead, 2 device task queue")
    ap.add_argument("--deterministic", type=int, default=1, choices=(0, 1),
                    help="1: fixed contribution order (the library default); 0: atomic order")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed-workload", default="elast27_48",
                    help="workload of the FP64 vs FP32+refinement comparison ('' to skip)")
    ap.add_argument("--mixed-steps", type=int, default=3)
    ap.add_argument("--batch", type=int, default=2000,
                    help="matrices of the batched workload (0 to skip)")
    ap.add_argument("--batch-options", default=None,
                    help="JSON dict of analysis options for the batched workload "
                         "(e.g. '{\"amalg_ratio\": 0.2}'), used as given, no tuning")
    ap.add_argument("--no-batch-tune", action="store_true",
                    help="batched workload with the default options (no amalgamation) "
                         "instead of the tuned ones")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the serving stream (0 to skip)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB (a dispatch of known traffic "
                         "for scaling hardware byte counters)")
    ap.add_argument("--cpu-batch-sample", type=int, default=2000,
                    help="matrices of the batched workload the oracle runs on a process "
                         "pool (0 to skip)")
    ap.add_argument("--cpu-sample", default=None,
                    help="grid of the bounded oracle sample (default: 44^3 for 3D workloads, "
                         "the full grid for 2D ones)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1608_00044_amd import inputs, spchol

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy_mib:
        src = torch.ones(args.calibrate_copy_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read, %d MiB written" % (args.calibrate_copy_mib,
                                                                  args.calibrate_copy_mib))
        del src, dst
    name = args.workload
    p = inputs.make_workload(name)
    amalg = p.meta["amalg"]
    log("workload", name, "n", p.n, "nnz", p.nnz)

    t0 = time.perf_counter()
    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=150, amalg_ratio=amalg,
                         sched=args.sched,
                         deterministic=args.deterministic if args.sched != 2 else 0)
    analyze_ms = (time.perf_counter() - t0) * 1e3
    info = sym.info()
    F = info["flops"]
    uflops = update_flops(sym)
    log("analyze %.1f ms, nsup %d, levels %d, F %.4e" % (analyze_ms, info["nsup"],
                                                          info["nlevels"], F))

    vals = torch.from_numpy(p.values).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(p.rhs[:, 0])).to(dev)
    stream = torch.cuda.current_stream()
    num = spchol.factor(sym, vals)
    st = num.status()
    if st != 0:
        raise RuntimeError("factor status %d" % st)
    x = num.solve(b)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        num.refactor(vals)
        num.solve(b, x=x)
    torch.cuda.synchronize()
    log("warmup done")

    # timed steps: the library as a caller uses it (no per-launch events)
    f_ms, s_ms = [], []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        e0, e1, e2 = ev[k]
        e0.record(stream)
        num.refactor(vals)
        e1.record(stream)
        num.solve(b, x=x)
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for e0, e1, e2 in ev:
        f_ms.append(e0.elapsed_time(e1))
        s_ms.append(e1.elapsed_time(e2))
    # per-kernel-class device time: separate factorizations with per-launch
    # events on the library's stream (launched directly, not from the graph)
    num.set_timing(True)
    kern = {c: 0.0 for c in spchol.KERNEL_CLASSES}
    launches = {c: 0 for c in spchol.KERNEL_CLASSES}
    kreps = max(2, min(args.steps, 5))
    for k in range(kreps):
        num.refactor(vals)
        tm = num.timing()  # synchronizes
        for c in spchol.KERNEL_CLASSES:
            kern[c] += tm[c]["ms"] / kreps * args.steps
            launches[c] += tm[c]["launches"] / kreps * args.steps
    num.set_timing(False)
    factor_ms = float(np.mean(f_ms))
    gflops = F / (factor_ms * 1e-3) / 1e9
    log("factor %.3f ms (min %.3f) -> %.1f GFLOP/s; kernels %s" %
        (factor_ms, min(f_ms), gflops, {c: round(kern[c] / args.steps, 3) for c in kern}))

    # solve latency: fresh N(0,1) right-hand sides, one solve at a time
    rng = np.random.Generator(np.random.PCG64(4242))
    nsol = args.solves
    B = torch.from_numpy(rng.standard_normal((nsol, p.n))).to(dev)
    lat = []
    for i in range(nsol):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        num.solve(B[i], x=x)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat = np.array(lat)
    xs = x.cpu().numpy()
    eta = backward_error(p, xs, B[nsol - 1].cpu().numpy())
    log("solve p50 %.3f ms p99 %.3f ms, backward error %.2e" %
        (np.percentile(lat, 50), np.percentile(lat, 99), eta))

    if args.sched == 2:
        # one persistent launch runs every F, T and U task of the factorization
        kname, kcls, kflops = ("k_sched (persistent task queue: POTRF, TRSM, FP64 MFMA update "
                               "tiles + scatter)", "tasks", F)
    else:
        kname, kcls, kflops = ("k_update (FP64 MFMA SYRK tile + relative-index scatter)",
                               "update", uflops)
    k_ms = kern[kcls] / args.steps
    k_launch = launches[kcls] / args.steps
    achieved = kflops / (k_ms * 1e-3) / 1e12 if k_ms > 0 else 0.0
    traffic = measured_traffic("k_update", name) if kcls == "update" else None
    roofline = {"kernel": kname,
                "bound": "mfma", "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "traffic": traffic,
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                "scaled by a copy kernel; profiles/)",
                "algorithmic_flops_per_launch": kflops / max(k_launch, 1),
                "avg_launch_ms": k_ms / max(k_launch, 1), "launches_per_factor": k_launch}

    hb = hbm_bytes(sym)
    p50 = float(np.percentile(lat, 50))
    hbm = {"peak_GBps": HBM_PEAK_GBPS,
           "solve": {"algorithmic_bytes": hb["solve"], "ms": p50,
                     "GBps": hb["solve"] / (p50 * 1e-3) / 1e9,
                     "frac": hb["solve"] / (p50 * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                     "note": "p50 single-RHS solve; latency bound (one launch pair per level)"},
           "scatter": {"algorithmic_bytes": hb["scatter"], "ms": kern["update"] / args.steps,
                       "GBps": hb["scatter"] / (kern["update"] / args.steps * 1e-3) / 1e9
                       if kern["update"] > 0 else 0.0,
                       "note": "scatter bytes over the whole update kernel time (fused with "
                               "the products): a lower bound on the scatter's own rate"}}
    hbm["scatter"]["frac"] = hbm["scatter"]["GBps"] / HBM_PEAK_GBPS
    out = {
        "metric": METRIC, "value": gflops, "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "description": WORKLOAD_TEXT.get(name, name), "n": p.n,
                   "nnz_lower": p.nnz, "nnz_L": info["nnz_l"], "flops_F": F,
                   "flops_stored": info["flops_stored"], "sn_cap": 150, "amalg_ratio": amalg,
                   "nsup": info["nsup"], "levels": info["nlevels"], "nrhs": 1,
                   "schedule": ["level sets", "level sets + lookahead",
                                "device task queue"][args.sched],
                   "precision": "fp64"},
        "factor_ms": factor_ms, "factor_ms_min": float(min(f_ms)),
        "solve_ms_in_step": float(np.mean(s_ms)),
        "solve_p50_ms": float(np.percentile(lat, 50)),
        "solve_p99_ms": float(np.percentile(lat, 99)),
        "solves_per_s": float(1e3 / np.mean(lat)),
        "solve_backward_error": eta, "analyze_ms": analyze_ms,
        "kernel_ms_per_factor": {c: kern[c] / args.steps for c in kern},
        "kernel_launches_per_factor": {c: launches[c] / args.steps for c in launches},
        "roofline": roofline,
        "hbm_phases": hbm,
    }
    num.free()
    sym.free()
    if args.mixed_workload:
        out["mixed_precision"] = mixed_precision(args.mixed_workload, args.mixed_steps, 1)
    if args.batch:
        tb = not args.no_batch_tune and not args.batch_options
        fixed = json.loads(args.batch_options) if args.batch_options else None
        out["batched"] = [batched(args.batch, 3, 0, tune_options=tb, options=fixed),
                          batched(args.batch, 3, 1, tune_options=tb, options=fixed)]
    if args.serve_requests:
        out["serving"] = serving(args.serve_requests)
    if not args.no_cpu_baseline:
        if args.cpu_sample:
            dims = tuple(int(v) for v in args.cpu_sample.split(","))
        else:
            full = inputs.WORKLOADS[name]["dims"]
            dims = (44, 44, 44) if len(full) == 3 else full
        log("cpu baseline on", dims)
        out["cpu_baseline"] = cpu_baseline(name, dims)
        if args.batch and args.cpu_batch_sample:
            log("cpu baseline of the batch, %d matrices" % min(args.batch, args.cpu_batch_sample))
            out["batched_cpu_baseline"] = cpu_batch_baseline(
                args.batch, min(args.batch, args.cpu_batch_sample))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
