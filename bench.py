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


class OracleLeg:
    """The CPU baseline: the oracle (plain left-looking column Cholesky, one
    core) on the whole workload, in a thread pinned to one host core while the
    GPU legs run (the oracle's C code releases the interpreter lock).  It
    factors (timed), then solves the workload's right-hand side; the small 2D
    workload (64 x 64) follows for its own parity check.  Nothing else of the
    benchmark calls the oracle: the parity of the GPU factor and solution is
    computed from this leg's results."""

    def __init__(self, name, small_name="lap2d_5pt_64"):
        import threading

        self.name, self.small_name = name, small_name
        self.result, self.error = None, None
        cores = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else [0]
        self.core = cores[-1]
        self.thread = threading.Thread(target=self._run, daemon=True)
        self.thread.start()

    def _run(self):
        try:
            try:
                os.sched_setaffinity(0, {self.core})  # this thread only
            except (AttributeError, OSError):
                pass
            import oracle
            from paper_1608_00044_amd import inputs

            out = {}
            for key, nm in (("main", self.name), ("small", self.small_name)):
                p = inputs.make_workload(nm)
                t0 = time.perf_counter()
                Cp, Ci, Cx, _ = oracle.permute(p.n, p.colptr, p.rowind, p.values, p.perm)
                sym = oracle.symbolic(p.n, Cp, Ci)
                t1 = time.perf_counter()
                st, Lx = oracle.factor(p.n, Cp, Ci, Cx, sym)
                t2 = time.perf_counter()
                if st != 0:
                    raise RuntimeError("oracle status %d on %s" % (st, nm))
                x = oracle.solve(p.n, sym, Lx, p.perm, p.rhs)
                t3 = time.perf_counter()
                out[key] = dict(n=p.n, C=(Cp, Ci, Cx), Lp=sym.Lp, Li=sym.Li, Lx=Lx, x=x,
                                flops=float(sym.flops), symbolic_s=t1 - t0, factor_s=t2 - t1,
                                solve_s=t3 - t2)
                log("oracle %s: symbolic %.1f s, factor %.1f s, solve %.1f s" %
                    (nm, t1 - t0, t2 - t1, t3 - t2))
            self.result = out
        except Exception as e:  # reported by join()
            self.error = e

    def join(self):
        self.thread.join()
        if self.error is not None:
            raise self.error
        return self.result


def factor_parity(n, Cp, Ci, Cx, Lp, Li, Lx, Sp, Si, Sx):
    """Element-by-element comparison of a GPU factor (stored structure
    Sp, Si, Sx) with the oracle's (exact structure Lp, Li, Lx): the worst
    |dL_ij| / (1e-10 |L_ij| + 1e-13 sqrt(c_ii c_jj) / L_jj) (c = the diagonal
    of P A P^T), the largest relative difference, and whether every stored
    entry outside the exact structure is an explicit zero."""
    ks = np.repeat(np.arange(n, dtype=np.int64), np.diff(Sp)) * n + Si
    ko = np.repeat(np.arange(n, dtype=np.int64), np.diff(Lp)) * n + Li
    pos = np.searchsorted(ks, ko)
    if not ((pos < ks.size).all() and np.array_equal(ks[pos], ko)):
        return {"entries": int(Lx.size), "structure_contained": False}
    del ko
    extra = np.ones(ks.size, dtype=bool)
    extra[pos] = False
    del ks
    got = Sx[pos]
    diag = np.zeros(n)
    nz = Cp[1:] > Cp[:-1]
    idx, js = Cp[:-1][nz], np.arange(n)[nz]
    isd = Ci[idx] == js
    diag[js[isd]] = Cx[idx[isd]]
    cols = np.repeat(np.arange(n), np.diff(Lp))
    ljj = Lx[Lp[:-1]][cols]
    tol = 1e-10 * np.abs(Lx) + 1e-13 * np.sqrt(np.abs(diag[Li] * diag[cols])) / np.abs(ljj)
    err = np.abs(got - Lx)
    return {"entries": int(Lx.size), "structure_contained": True,
            "explicit_zeros_ok": bool((Sx[extra] == 0.0).all()),
            "worst_over_tolerance": float((err / tol).max()),
            "max_rel_diff": float((err / np.maximum(np.abs(Lx), 1e-300)).max()),
            "bar": "|dL_ij| <= 1e-10 |L_ij| + 1e-13 sqrt(c_ii c_jj) / L_jj for every entry"}


def probe_residual(p, Sp, Si, Sx, probes=8, seed=7):
    """rho ~ ||(L L^T - P A P^T) Z||_F / ||P A P^T Z||_F over `probes` N(0,1)
    columns (an unbiased estimate of ||L L^T - P A P^T||_F / ||P A P^T||_F up to
    the probes' spread), from a factor on the host (scipy; no oracle)."""
    import scipy.sparse as sp

    A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
    A = (A + sp.tril(A, -1).T).tocsr()
    perm = p.perm if p.perm is not None else np.arange(p.n)
    C = A[perm][:, perm]
    L = sp.csc_matrix((Sx, Si, Sp), shape=(p.n, p.n))
    Z = np.random.default_rng(seed).standard_normal((p.n, probes))
    CZ = C @ Z
    R = L @ (L.T @ Z) - CZ
    return float(np.linalg.norm(R) / np.linalg.norm(CZ))


def exact_residual(p, Sp, Si, Sx):
    """||L L^T - P A P^T||_F / ||A||_F exactly (scipy sparse products)."""
    import scipy.sparse as sp

    A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
    A = (A + sp.tril(A, -1).T).tocsr()
    perm = p.perm if p.perm is not None else np.arange(p.n)
    C = A[perm][:, perm]
    L = sp.csc_matrix((Sx, Si, Sp), shape=(p.n, p.n))
    D = (L @ L.T - C).tocoo()
    return float(np.sqrt((D.data ** 2).sum()) / sp.linalg.norm(A))


def stored_oracle_solution(name):
    """The FP64 oracle's solution of `name` stored under tests/golden/ by
    tests/golden/make_oracle_solution.py (read here with numpy only), or None
    when absent or written by other sources of the oracle or the inputs."""
    import hashlib

    path = os.path.join(ROOT, "tests", "golden", "oracle_x_%s.npz" % name)
    if not os.path.exists(path):
        return None
    want = {}
    for key, rel in (("oracle_sha", "oracle/oracle.c"),
                     ("inputs_sha", "paper_1608_00044_amd/inputs.py")):
        with open(os.path.join(ROOT, rel), "rb") as f:
            want[key] = hashlib.sha256(f.read()).hexdigest()
    with np.load(path, allow_pickle=False) as z:
        if any(str(z[k]) != v for k, v in want.items()) or str(z["workload"]) != name:
            return None
        return np.array(z["x"]), np.array(z["eta"])


def oracle_factor_parity(name, p, Sp, Si, Sx):
    """Worst |dL_ij| / (1e-10 |L_ij| + 1e-13 sqrt(c_ii c_jj) / |L_jj|) of the GPU
    factor over the FP64 oracle's factor entries stored under tests/golden/ by
    tests/golden/make_oracle_factor_sample.py (every stride-th entry of the
    exact structure; read here with numpy only), with C = P A P^T; None when
    the sample is absent or written by other sources of the oracle or the
    inputs."""
    import hashlib

    path = os.path.join(ROOT, "tests", "golden", "oracle_L_sample_%s.npz" % name)
    if not os.path.exists(path):
        return None
    want = {}
    for key, rel in (("oracle_sha", "oracle/oracle.c"),
                     ("inputs_sha", "paper_1608_00044_amd/inputs.py")):
        with open(os.path.join(ROOT, rel), "rb") as f:
            want[key] = hashlib.sha256(f.read()).hexdigest()
    with np.load(path, allow_pickle=False) as z:
        if any(str(z[k]) != v for k, v in want.items()) or str(z["workload"]) != name:
            return None
        rows, cols, ref, ljj = (np.array(z[k]) for k in ("rows", "cols", "vals", "ljj"))
        stride, nnz_l = int(z["stride"]), int(z["nnz_l"])
    n = p.n
    colA = np.repeat(np.arange(n), np.diff(p.colptr))
    isd = p.rowind == colA
    diagA = np.zeros(n)
    diagA[colA[isd]] = p.values[isd]
    perm = p.perm if p.perm is not None else np.arange(n)
    c = diagA[perm]
    # binary search of each sampled row in its column (rows increase within
    # a stored column)
    lo, end = Sp[cols].astype(np.int64), Sp[cols + 1].astype(np.int64)
    hi = end.copy()
    while (lo < hi).any():
        act = lo < hi
        mid = (lo + hi) // 2
        go = Si[np.minimum(mid, Si.size - 1)] < rows
        lo = np.where(act & go, mid + 1, lo)
        hi = np.where(act & ~go, mid, hi)
    if (lo >= end).any() or (Si[np.minimum(lo, Si.size - 1)] != rows).any():
        return {"worst": float("inf"), "what": "oracle entry outside the stored structure"}
    pos = lo
    bar = 1e-10 * np.abs(ref) + 1e-13 * np.sqrt(np.abs(c[rows] * c[cols])) / np.abs(ljj)
    worst = float((np.abs(Sx[pos] - ref) / bar).max())
    return {"worst": worst, "entries": int(ref.size), "of": nnz_l, "stride": stride,
            "what": "max |L_gpu - L_oracle| / (1e-10 |L| + 1e-13 sqrt(c_ii c_jj) / |L_jj|) "
                    "over every %d-th entry of the oracle's exact factor "
                    "(tests/golden/oracle_L_sample_%s.npz); <= 1 passes" % (stride, name)}


def other_order(p, amalg, F, deterministic, steps, primary_ms):
    """The workload factored in the other contribution order (deterministic
    or atomic), timed the same way; its cost against the headline order."""
    import torch

    from paper_1608_00044_amd import spchol

    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=150, amalg_ratio=amalg,
                         deterministic=deterministic)
    vals = torch.from_numpy(p.values).to("cuda:0")
    b = torch.from_numpy(np.ascontiguousarray(p.rhs[:, 0])).to("cuda:0")
    num = spchol.factor(sym, vals)
    if num.status() != 0:
        raise RuntimeError("factor status %d" % num.status())
    x = num.solve(b)
    stream = torch.cuda.current_stream()
    f_ms, s_ms = [], []
    for k in range(steps + 1):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        num.refactor(vals)
        e1.record(stream)
        num.solve(b, x=x)
        e2.record(stream)
        torch.cuda.synchronize()
        if k:
            f_ms.append(e0.elapsed_time(e1))
            s_ms.append(e1.elapsed_time(e2))
    fm = float(np.mean(f_ms))
    out = {"deterministic": deterministic,
           "order": "fixed (bitwise reproducible)" if deterministic else "atomic",
           "factor_ms": fm, "factor_gflops": F / (fm * 1e-3) / 1e9,
           "solve_ms": float(np.mean(s_ms)),
           "factor_time_ratio_to_headline": fm / primary_ms}
    log("other order (deterministic=%d): factor %.3f ms (%.3fx)" % (deterministic, fm,
                                                                     fm / primary_ms))
    num.free()
    sym.free()
    return out


def small_workload(name, solves):
    """The latency-bound 2D workload (64 x 64 grid): factor time (HIP events),
    solve p50/p99 over `solves` fresh right-hand sides, backward error, the
    exact residual; returns (report, the factor's export for oracle parity)."""
    import torch

    from paper_1608_00044_amd import inputs, spchol

    p = inputs.make_workload(name)
    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=150, amalg_ratio=p.meta["amalg"])
    inf = sym.info()
    vals = torch.from_numpy(p.values).to("cuda:0")
    b = torch.from_numpy(np.ascontiguousarray(p.rhs[:, 0])).to("cuda:0")
    num = spchol.factor(sym, vals)
    if num.status() != 0:
        raise RuntimeError("factor status %d" % num.status())
    x = num.solve(b)
    stream = torch.cuda.current_stream()
    f_us = []
    for k in range(21):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        num.refactor(vals)
        e1.record(stream)
        torch.cuda.synchronize()
        if k:
            f_us.append(e0.elapsed_time(e1) * 1e3)
    rng = np.random.Generator(np.random.PCG64(4243))
    Bm = torch.from_numpy(rng.standard_normal((solves, p.n))).to("cuda:0")
    lat = []
    for i in range(solves):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        num.solve(Bm[i], x=x)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e6)
    x = num.solve(b).cpu().numpy()
    eta = backward_error(p, x, p.rhs[:, 0])
    Sp, Si, Sx = num.export()
    rho = exact_residual(p, Sp, Si, Sx)
    out = {"workload": name, "description": WORKLOAD_TEXT.get(name, name), "n": p.n,
           "nnz_L": inf["nnz_l"], "flops_F": inf["flops"], "nsup": inf["nsup"],
           "levels": inf["nlevels"], "factor_us": float(np.mean(f_us)),
           "factor_gflops": inf["flops"] / (np.mean(f_us) * 1e-6) / 1e9,
           "solve_p50_us": float(np.percentile(lat, 50)),
           "solve_p99_us": float(np.percentile(lat, 99)),
           "backward_error": eta, "residual_exact": rho,
           "bound": "latency (launches per level); roofline fractions near zero"}
    log("small 2D: factor %.1f us, solve p50 %.1f us p99 %.1f us, eta %.1e, rho %.1e" %
        (out["factor_us"], out["solve_p50_us"], out["solve_p99_us"], eta, rho))
    num.free()
    sym.free()
    return out, (Sp, Si, Sx)


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
    robin): matrices/s over the pool's wall time (spawn included), beside the
    one-core sum and the makespan (the slowest worker's summed compute time)."""
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
    return {"value": sample / wall, "unit": "matrices/s", "cores": workers, "kind": "oracle",
            "sample": "first %d of the %d matrices: permute + symbolic + factor + one-RHS "
                      "solve each; %d worker processes, members dealt round robin"
                      % (sample, count, workers),
            "one_core_sum_s": one_core, "makespan_s": makespan, "pool_wall_s": wall,
            "one_core_matrices_per_s": sample / one_core,
            "makespan_matrices_per_s": sample / makespan,
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


def mixed_precision(name, steps, warmup, tol=1e-10, deterministic=0):
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
    ref = stored_oracle_solution(name)
    if ref is not None:
        import scipy.sparse as sp

        A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
        A = A + sp.tril(A, -1).T
        # lambda_min >= the diagonal shift (the edge blocks form a positive
        # semidefinite operator), so cond(A) <= ||A||_inf / shift
        kappa = float(abs(A).sum(axis=1).max()) / p.meta["shift"]
        out["fp64_oracle_solution"] = {
            "source": "tests/golden/oracle_x_%s.npz: the FP64 oracle's solution of all %d "
                      "right-hand sides, written once by tests/golden/make_oracle_solution.py "
                      "(keyed by the SHA-256 of oracle/oracle.c and the input generator)"
                      % (name, k),
            "oracle_backward_error": float(np.max(ref[1])), "cond_bound": kappa}
    for prec in (0, 1):
        sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=150,
                             amalg_ratio=p.meta["amalg"], precision=prec,
                             deterministic=deterministic)
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
        if ref is not None:
            xo, eta_o = ref
            xo = xo.reshape(p.n, -1)
            err = max(float(np.abs(xs[:, c] - xo[:, c]).max() / np.abs(xo[:, c]).max())
                      for c in range(k))
            out[key]["error_vs_fp64_oracle"] = err
            out[key]["error_bound"] = 4.0 * out["fp64_oracle_solution"]["cond_bound"] * (
                eta + float(np.max(eta_o)))
            log("  %s error vs the FP64 oracle's solution %.2e (bound %.2e)" %
                (key, err, out[key]["error_bound"]))
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


TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1608_00044_amd",
                          "tuned_batch.json")


def batched(count, steps, precision, tol=1e-10, tune_options=True, options=None,
            deterministic=0, launch_form_sample=200, retune=False, cache=TUNE_CACHE):
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
    base = dict(tune.BASE, deterministic=deterministic)
    opts, table, tuned = dict(base, **(options or {})), None, None
    if tune_options:
        t0 = time.perf_counter()
        opts, table = tune.tune_batch(mats, vals, b, precision, base=base,
                                      cache_path=cache, retune=retune)
        tuned = "timed in this run" if table is not None else \
            "cached choice of an earlier timed run (%s)" % os.path.basename(cache)
        if table is None:
            table = tune.cached_table(mats, precision, cache)
        log("batch tuning (%.1f s, %s): %s" % (time.perf_counter() - t0, tuned, opts))
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
        out["tuning"] = [dict(t["options"], stage=t["stage"], ms=t["ms"], nsup=t.get("nsup"),
                              levels=t.get("levels")) for t in table]
        out["tuning_source"] = tuned
    if precision == 1:
        out["refine_iters"] = float(np.mean(iters))
    log("batch %s: factor %.2f ms (%.1f GFLOP/s), solve %.2f ms, %.0f matrices/s" %
        (out["precision"], fm, out["factor_gflops"], sm, out["matrices_per_s"]))
    num.free()
    sym.free()
    if precision == 0 and launch_form_sample > 0:
        out["launch_forms"] = launch_forms(mats[:launch_form_sample],
                                           vals[:sum(int(m[1][int(m[0])]) for m in
                                                     mats[:launch_form_sample])],
                                           opts, steps)
    return out


def launch_forms(mats, vals, opts, steps):
    """The batch's factorization in its two launch forms on the same members
    and options: level-set launches over all matrices at once (sched 0, the
    lane-group kernels for small supernodes) against one persistent
    task-queue launch (sched 2, Section IV's counters; every supernode a
    workgroup task, atomic contribution order)."""
    import torch

    from paper_1608_00044_amd import spchol

    res = {"matrices": len(mats)}
    for name, extra in (("level_sets", dict(sched=0, deterministic=0)),
                        ("task_queue", dict(sched=2, deterministic=0))):
        t0 = time.perf_counter()
        sym = spchol.analyze_batch(mats, **dict(opts, **extra))
        num = spchol.factor(sym, vals)
        torch.cuda.synchronize()
        prep = time.perf_counter() - t0
        if num.status() != 0:
            raise RuntimeError("%s factor status %d" % (name, num.status()))
        ms = []
        for _ in range(max(1, steps)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            num.refactor(vals)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        res[name + "_factor_ms"] = float(np.mean(ms))
        res[name + "_setup_s"] = prep
        num.free()
        sym.free()
    res["winner"] = min(("level_sets", "task_queue"), key=lambda k: res[k + "_factor_ms"])
    log("batch launch forms on %d matrices: level sets %.2f ms, task queue %.2f ms" %
        (len(mats), res["level_sets_factor_ms"], res["task_queue_factor_ms"]))
    return res


SERVE_RECIPE = dict(rate=200.0, patterns_2d=16, patterns_3d=16, side2d=(32, 256),
                    side3d=(16, 48), sigma=1.0, solve_only=0.3, nrhs=(1, 4, 16, 64),
                    value_sets=2)


def serving(requests, seed=5000, deterministic=0):
    """Poisson request stream over 32 resident patterns through the request
    server; reports latency percentiles and throughput (patterns analysed in
    the given contribution order)."""
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
    syms = [spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=150, amalg_ratio=0.1,
                           deterministic=deterministic) for p in probs]
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
    que = np.array([q["queue_ms"] for q in res])
    # each pattern's first request also makes its first factor (allocation
    # and the capture of its launch graphs)
    first = np.zeros(requests, dtype=bool)
    seen_p = set()
    for i in range(requests):
        if pat[i] not in seen_p:
            first[i] = True
            seen_p.add(pat[i])
    run = lat - que  # admission to completion of the request's device work
    ok = sum(1 for q in res if q["status"] == 0)
    cols = int(sum(int(nrhs[i]) for i in range(requests) if res[i]["status"] == 0))
    out = {"requests": requests, "rate_per_s": r["rate"], "patterns": len(probs),
           "ok": ok, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "requests_per_s": requests / wall,
           "queue_p50_ms": float(np.percentile(que, 50)),
           "queue_p99_ms": float(np.percentile(que, 99)),
           "admitted_p50_ms": float(np.percentile(run, 50)),
           "admitted_p99_ms": float(np.percentile(run, 99)),
           "warm_p50_ms": float(np.percentile(lat[~first], 50)),
           "warm_p99_ms": float(np.percentile(lat[~first], 99)),
           "first_request_p50_ms": float(np.percentile(lat[first], 50)),
           "first_request_max_ms": float(lat[first].max()),
           "latency_split": "latency = queue (submission to admission: waiting for a slot, "
                            "memory or a factor) + admitted (admission to the end of the "
                            "request's device work, overlapping other requests)",
           "order": "fixed (bitwise reproducible)" if deterministic else "atomic",
           "solves_per_s": cols / wall, "peak_inflight": st["peak_inflight"],
           "peak_bytes": st["peak_bytes"], "evictions": st["evictions"],
           "recipe": "Poisson arrivals at %g/s over %d 2D (side %d..%d) and %d 3D 7-point "
                     "(side %d..%d) patterns, lognormal(0,%g) weights, %d%% solve-only on the "
                     "current factor, nrhs uniform in %s" % (
                         r["rate"], r["patterns_2d"], r["side2d"][0], r["side2d"][1],
                         r["patterns_3d"], r["side3d"][0], r["side3d"][1], r["sigma"],
                         int(100 * r["solve_only"]), list(r["nrhs"]))}
    log("serve: p50 %.2f ms p99 %.2f ms (warm %.2f / %.2f, first requests p50 %.2f ms), "
        "%.1f req/s, %.0f solves/s, peak inflight %d" %
        (out["p50_ms"], out["p99_ms"], out["warm_p50_ms"], out["warm_p99_ms"],
         out["first_request_p50_ms"], out["requests_per_s"], out["solves_per_s"],
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
    ap.add_argument("--deterministic", type=int, default=0, choices=(0, 1),
                    help="contribution order of the timed factorization: 0 atomic (default "
                         "here), 1 fixed (bitwise reproducible; the library default); the "
                         "other order is timed beside it")
    ap.add_argument("--other-order-steps", type=int, default=5,
                    help="timed factorizations in the other contribution order (0 to skip)")
    ap.add_argument("--small-workload", default="lap2d_5pt_64",
                    help="the latency-bound 2D workload reported beside ('' to skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed-workload", default="elast27_48",
                    help="workload of the FP64 vs FP32+refinement comparison ('' to skip)")
    ap.add_argument("--mixed-steps", type=int, default=3)
    ap.add_argument("--batch", type=int, default=2000,
                    help="matrices of the batched workload (0 to skip)")
    ap.add_argument("--batch-options", default=None,
                    help="JSON dict of analysis options for the batched workload "
                         "(e.g. '{\"amalg_ratio\": 0.2}'), used as given, no tuning")
    ap.add_argument("--retune", action="store_true",
                    help="time the batch autotuner's candidates again and store the "
                         "choices in paper_1608_00044_amd/tuned_batch.json (default: "
                         "use the stored choice of the batch's size class, if any)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="the autotuner's JSON cache of choices per size class")
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
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    leg = None
    if not args.no_cpu_baseline:
        # the oracle on the whole workload, in a thread on one host core of its
        # own beside the GPU legs (this thread and its children keep off that core)
        leg = OracleLeg(args.workload, args.small_workload or "lap2d_5pt_64")
        try:
            others = set(os.sched_getaffinity(0)) - {leg.core}
            if others:
                os.sched_setaffinity(0, others)
        except (AttributeError, OSError):
            pass

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
    # the workload's own right-hand side and the factor, for parity with the
    # oracle (CPU-baseline leg) and the probe residual
    x_main = num.solve(b).cpu().numpy()
    Sp, Si, Sx = num.export()
    rho = probe_residual(p, Sp, Si, Sx)
    log("probe residual %.2e" % rho)
    lpar = oracle_factor_parity(name, p, Sp, Si, Sx)
    if lpar is not None:
        log("factor vs stored oracle entries: worst %.3g of the bar over %d entries" %
            (lpar["worst"], lpar.get("entries", 0)))
    log("solve p50 %.3f ms p99 %.3f ms, backward error %.2e" %
        (np.percentile(lat, 50), np.percentile(lat, 99), eta))

    if args.sched == 2:
        # one persistent launch runs every F, T and U task of the factorization
        kname, kcls, kflops = ("k_sched (persistent task queue: POTRF, TRSM, FP64 MFMA update "
                               "tiles + scatter)", "tasks", F)
    else:
        kname, kcls, kflops = ("k_update (FP64 MFMA SYRK tile + relative-index scatter; %s "
                               "contribution order)" % ("fixed" if args.deterministic else
                                                        "atomic"), "update", uflops)
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

    ceil = spchol.measure_ceilings()
    log("measured ceilings: %s" % ceil)
    roofline["measured_ceiling"] = ceil["fp64_mfma_tflops"]
    roofline["frac_of_measured_ceiling"] = achieved / ceil["fp64_mfma_tflops"]
    hb = hbm_bytes(sym)
    p50 = float(np.percentile(lat, 50))
    hbm = {"peak_GBps": HBM_PEAK_GBPS,
           "solve": {"algorithmic_bytes": hb["solve"], "ms": p50,
                     "GBps": hb["solve"] / (p50 * 1e-3) / 1e9,
                     "frac": hb["solve"] / (p50 * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                     "note": "p50 single-RHS solve; latency bound (one launch per level and direction, plus the forward's shared-row reductions)"},
           "scatter": {"algorithmic_bytes": hb["scatter"], "ms": kern["update"] / args.steps,
                       "GBps": hb["scatter"] / (kern["update"] / args.steps * 1e-3) / 1e9
                       if kern["update"] > 0 else 0.0,
                       "note": "scatter bytes over the whole update kernel time (fused with "
                               "the products): a lower bound on the scatter's own rate"}}
    hbm["scatter"]["frac"] = hbm["scatter"]["GBps"] / HBM_PEAK_GBPS
    hbm["measured_copy_GBps"] = ceil["copy_gbs"]
    for k in ("solve", "scatter"):
        hbm[k]["frac_of_measured_copy"] = hbm[k]["GBps"] / ceil["copy_gbs"]
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
        "measured_ceilings": dict(ceil, what="spc_measure_ceilings: 16x16x4 matrix-core "
                                                "products from registers (8 accumulators per "
                                                "wave, 8 waves per SIMD) and a 512 MiB copy "
                                                "(read + write bytes)"),
        "oracle_sample_parity": lpar,
        "residual_probe": {"value": rho, "probes": 8,
                           "what": "||(L L^T - P A P^T) Z||_F / ||P A P^T Z||_F, Z 8 N(0,1) "
                                   "columns, GPU factor on the host (scipy)"},
    }
    num.free()
    sym.free()
    if args.other_order_steps and args.sched != 2:
        out["other_order"] = other_order(p, amalg, F, 1 - args.deterministic,
                                         args.other_order_steps, factor_ms)
    small_export = None
    if args.small_workload:
        out["small_2d"], small_export = small_workload(args.small_workload, args.solves)
    if args.mixed_workload:
        out["mixed_precision"] = mixed_precision(args.mixed_workload, args.mixed_steps, 1,
                                                 deterministic=args.deterministic)
    if args.batch:
        tb = not args.no_batch_tune and not args.batch_options
        fixed = json.loads(args.batch_options) if args.batch_options else None
        out["batched"] = [batched(args.batch, 3, prec, tune_options=tb, options=fixed,
                                  deterministic=args.deterministic, retune=args.retune,
                                  cache=args.tune_cache)
                          for prec in (0, 1)]
    if args.serve_requests:
        out["serving"] = serving(args.serve_requests, deterministic=args.deterministic)
    if leg is not None:
        log("waiting for the oracle leg")
        res = leg.join()
        m = res["main"]
        out["cpu_baseline"] = {
            "value": m["flops"] / m["factor_s"] / 1e9, "unit": "GFLOP/s", "cores": 1,
            "kind": "oracle",
            "sample": "the whole %s workload (n=%d, F=%.4e): the oracle's numeric "
                      "factorization (plain left-looking column Cholesky, untuned) on one "
                      "pinned host core, %.1f s, run in a thread beside the GPU legs; "
                      "symbolic %.1f s and solve %.1f s not counted"
                      % (name, m["n"], m["flops"], m["factor_s"], m["symbolic_s"], m["solve_s"])}
        par = factor_parity(m["n"], *m["C"], m["Lp"], m["Li"], m["Lx"], Sp, Si, Sx)
        xo = np.asarray(m["x"]).reshape(p.n, -1)[:, 0]
        par["solution_max_rel_diff"] = float(np.abs(x_main - xo).max() / np.abs(xo).max())
        out["oracle_parity"] = par
        log("oracle parity: %s" % par)
        if small_export is not None:
            sm = res["small"]
            sp_ = factor_parity(sm["n"], *sm["C"], sm["Lp"], sm["Li"], sm["Lx"], *small_export)
            out["small_2d"]["oracle_parity"] = sp_
        del res, m
        if args.batch and args.cpu_batch_sample:
            log("cpu baseline of the batch, %d matrices" % min(args.batch, args.cpu_batch_sample))
            out["batched_cpu_baseline"] = cpu_batch_baseline(
                args.batch, min(args.batch, args.cpu_batch_sample))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
