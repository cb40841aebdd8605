"""Autotuner for batched factorization.

A batch of many small matrices is latency bound: one factorization is one
launch per kernel class per level of the batch's elimination forest, and
its cost follows the number of levels and of supernodes more than the flop
count.  Three choices move it, and the best setting depends on the
matrices' size and sparsity:
- the relaxed-amalgamation ratio (explicit zeros traded for fewer, wider
  supernodes and fewer levels);
- the supernode cap;
- which supernodes run on the lane-group kernels (16, 32 or 64 lanes per
  supernode, several supernodes per wave) and which on the workgroup
  kernels over 64 x 64 tiles (the small_w / small_r limits);
- the update tiles' shape: the columns of the source panel staged through
  LDS per step (8, 16 or 32: fewer steps against less LDS, and so more
  tiles resident per CU).
The tuner searches them one stage at a time (each stage starting from the
best options so far), timing every option set on the GPU through the
library's own entry points: one factorization plus one solve (FP64) or one
refined solve (FP32 factor).  Choices are cached in a JSON file keyed by a
size class of the batch (precision, count, mean order and mean entries per
column, each rounded to a coarse class), so later batches of the same class
reuse them without timing again.

Every option set computes the same factorization of the same matrices; only
the supernode partition (and so the explicit zeros stored) and the kernels
that run each supernode differ.
"""
from __future__ import annotations

import json
import math
import os
import time

from .spchol import SpcError

BASE = dict(amalg_ratio=0.0, sn_cap=150, small_w=16, small_r=64, upd_chunk=16)
STAGES = (
    tuple(dict(amalg_ratio=r) for r in (0.0, 0.05, 0.1, 0.2, 0.3, 0.5)),
    tuple(dict(sn_cap=c) for c in (150, 64)),
    tuple(dict(small_w=w, small_r=r)
          for w, r in ((16, 64), (16, 32), (8, 64), (4, 16), (-1, 64))),
    tuple(dict(upd_chunk=c) for c in (16, 8, 32)),
)


def size_class(mats, precision: int) -> str:
    """Cache key of a batch: precision, count (power of two), mean order
    (power of two) and mean stored lower entries per column (halves)."""
    count = len(mats)
    n = sum(int(m[0]) for m in mats)
    nnz = sum(int(m[1][int(m[0])]) for m in mats if int(m[0]) > 0)
    pow2 = (lambda v: 0 if v < 1 else 1 << int(round(math.log2(v))))
    deg = round(2.0 * nnz / n) / 2.0 if n else 0.0
    return "p%d-count%d-n%d-deg%g" % (precision, pow2(count), pow2(n / max(count, 1)), deg)


def measure(mats, values, rhs, precision, opts, steps=2, tol=1e-10):
    """Mean ms of factorization + solve (FP64) or factorization + refined
    solve to `tol` (FP32) on the current GPU, after one untimed step that
    builds the plan and captures the graphs.  `values` and `rhs` are device
    tensors (rhs one column per matrix, stacked)."""
    import torch

    from . import spchol

    sym = spchol.analyze_batch(mats, precision=precision, **opts)
    inf = sym.info()
    num = spchol.factor(sym, values)
    try:
        if num.status() != 0:
            raise spchol.SpcError(num.status(), "spc_factor")
        x = None
        ms = []
        for k in range(steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            num.refactor(values)
            if precision == 0:
                x = num.solve(rhs, x=x)
            else:
                x, _, _ = num.solve_refine(rhs, x=x, tol=tol, max_iter=20)
            torch.cuda.synchronize()
            if k > 0:
                ms.append((time.perf_counter() - t0) * 1e3)
        return {"ms": sum(ms) / len(ms), "nsup": inf["nsup"], "levels": inf["nlevels"],
                "flops_stored": inf["flops_stored"]}
    finally:
        num.free()
        sym.free()


def _load(path):
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return data if isinstance(data, dict) else {}


def _store(path, data):
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = "%s.tmp%d" % (path, os.getpid())
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached_table(mats, precision, cache_path):
    """The timed table stored with a cached choice (None if there is none)."""
    got = _load(cache_path).get(size_class(mats, precision))
    return None if got is None else got.get("table")


def tune_batch(mats, values, rhs, precision=0, stages=STAGES, cache_path=None, steps=2,
               timer=measure, base=BASE, retune=False):
    """Options (a dict for spchol.analyze_batch) that minimise factorization +
    solve time for this batch, and the table of what each timed option set
    measured.  A cached choice for the batch's size class is returned without
    timing (table None) unless `retune`.  Otherwise each stage's candidates (partial option
    dicts) are applied in turn to the best options so far and timed with
    `timer` (an option set already timed is not timed again; one that
    fails with a library error is recorded with ms = inf and never chosen);
    when `cache_path` is given, the winner is stored there."""
    key = size_class(mats, precision)
    cached = _load(cache_path).get(key)
    if cached is not None and not retune:
        return dict(cached["options"]), None
    best = dict(base)
    seen, table = {}, []
    for k, stage in enumerate(stages):
        for upd in stage:
            opts = dict(best, **upd)
            sig = tuple(sorted(opts.items()))
            if sig not in seen:
                try:
                    r = timer(mats, values, rhs, precision, dict(opts), steps=steps)
                except SpcError as e:  # e.g. refinement that does not converge
                    r = {"ms": math.inf, "error": e.status}
                seen[sig] = r["ms"]
                table.append(dict(options=opts, stage=k, **r))
        done = [t for t in table if math.isfinite(t["ms"])]
        if not done:
            raise RuntimeError("no candidate option set completed: %s" % table)
        best = dict(min(done, key=lambda t: t["ms"])["options"])
    if cache_path:
        data = _load(cache_path)
        data[key] = {"options": best, "ms": seen[tuple(sorted(best.items()))], "table": table}
        _store(cache_path, data)
    return best, table
