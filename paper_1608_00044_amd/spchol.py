"""Python binding of the spchol C ABI (include/spchol.h).

Argument marshalling only: every step of the factorization and solve runs in
the HIP library ``libspchol.so`` built in-tree by ``paper_1608_00044_amd.build``.
There is no fallback: if the library is missing, ``lib()`` raises.

Host arrays are numpy; device arrays are torch tensors on the current HIP
device (float64), passed by ``data_ptr()``; the stream is torch's current
stream unless one is given.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspchol.so")
_lib = None

SPC_OK = 0
SPC_ERR_ARG = -1
SPC_ERR_PATTERN = -2
SPC_ERR_OOM = -3
SPC_ERR_HIP = -4
SPC_ERR_NOT_FACTORED = -5
SPC_ERR_NOT_CONVERGED = -6
SPC_ERR_TIMEOUT = -7
SPC_ERR_BUSY = -8
SPC_ERR_TOO_LARGE = -9

# Every symbol include/spchol.h declares.
EXPORTS = ("spc_default_options", "spc_analyze", "spc_symbolic_info_get", "spc_symbolic_export",
           "spc_symbolic_export_rows", "spc_symbolic_export_pairs", "spc_symbolic_export_tasks",
           "spc_symbolic_free",
           "spc_factor", "spc_refactor", "spc_numeric_status", "spc_solve", "spc_factor_export",
           "spc_numeric_free", "spc_status_string", "spc_numeric_set_timing",
           "spc_numeric_get_timing", "spc_solve_refine", "spc_numeric_info_get",
           "spc_analyze_batch", "spc_server_default_options", "spc_server_create",
           "spc_server_add_pattern", "spc_server_submit", "spc_server_wait",
           "spc_server_stats_get", "spc_server_destroy", "spc_numeric_task_log",
           "spc_solve_noalloc", "spc_measure_ceilings")


class spc_options(C.Structure):
    _fields_ = [("sn_cap", C.c_int32), ("sched", C.c_int32), ("amalg_ratio", C.c_double),
                ("mem_budget_bytes", C.c_int64), ("spin_limit", C.c_int64),
                ("debug_flags", C.c_int32), ("precision", C.c_int32), ("threads", C.c_int32),
                ("small_w", C.c_int32), ("small_r", C.c_int32), ("deterministic", C.c_int32),
                ("workers", C.c_int32), ("solve_tail", C.c_int32), ("upd_chunk", C.c_int32)]


class spc_symbolic_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz_a", C.c_int64), ("nnz_l", C.c_int64),
                ("nnz_stored", C.c_int64), ("nsup", C.c_int64), ("nlevels", C.c_int64),
                ("npairs", C.c_int64), ("nrel", C.c_int64), ("factor_bytes", C.c_int64),
                ("plan_bytes", C.c_int64), ("flops", C.c_double), ("flops_stored", C.c_double),
                ("max_width", C.c_int32), ("max_below", C.c_int32), ("nbatch", C.c_int64),
                ("solve_bytes_per_rhs", C.c_int64), ("tail_levels", C.c_int32),
                ("tail_supernodes", C.c_int32)]


class spc_numeric_info(C.Structure):
    _fields_ = [("precision", C.c_int32), ("sched", C.c_int32), ("factor_bytes", C.c_int64),
                ("fp64_blocks", C.c_int64), ("refine_fallbacks", C.c_int64)]


class spc_server_options(C.Structure):
    _fields_ = [("max_inflight", C.c_int32), ("max_nrhs", C.c_int32),
                ("mem_budget_bytes", C.c_int64)]


class spc_request(C.Structure):
    _fields_ = [("pattern", C.c_int32), ("kind", C.c_int32), ("nrhs", C.c_int32),
                ("reserved", C.c_int32), ("values", C.c_void_p), ("b", C.c_void_p),
                ("ldb", C.c_int64), ("x", C.c_void_p), ("ldx", C.c_int64),
                ("stream", C.c_void_p)]


class spc_request_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_int32), ("queue_ms", C.c_double),
                ("latency_ms", C.c_double)]


class spc_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("evictions", C.c_int64), ("bytes_in_use", C.c_int64), ("peak_bytes", C.c_int64),
                ("budget_bytes", C.c_int64), ("peak_inflight", C.c_int32),
                ("resident_factors", C.c_int32)]


class spc_ceilings(C.Structure):
    _fields_ = [("fp64_mfma_tflops", C.c_double), ("fp32_mfma_tflops", C.c_double),
                ("copy_gbs", C.c_double)]


class spc_kernel_times(C.Structure):
    _fields_ = [("ms", C.c_double * 6), ("launches", C.c_int64 * 6), ("total_ms", C.c_double)]


KERNEL_CLASSES = ("load", "potrf", "trsm", "update", "tasks", "small")


class SpcError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = int(status)
        super().__init__("%s: %s (%d)" % (where, status_string(status), status))


def lib():
    """Load libspchol.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libspchol.so is not built; run paper_1608_00044_amd.build.build()")
        # torch ships its own HIP runtime: load it first so that the library
        # binds to that same runtime (one runtime per process, shared streams)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.spc_default_options.argtypes = [C.POINTER(spc_options)]
        L.spc_default_options.restype = None
        L.spc_analyze.argtypes = [C.c_int64, vp, vp, vp, C.POINTER(spc_options), C.POINTER(vp)]
        L.spc_analyze.restype = C.c_int32
        L.spc_analyze_batch.argtypes = [C.c_int32, vp, vp, vp, vp, C.POINTER(spc_options),
                                        C.POINTER(vp)]
        L.spc_analyze_batch.restype = C.c_int32
        L.spc_symbolic_info_get.argtypes = [vp, C.POINTER(spc_symbolic_info)]
        L.spc_symbolic_info_get.restype = C.c_int32
        L.spc_symbolic_export.argtypes = [vp, vp, vp, vp, vp]
        L.spc_symbolic_export.restype = C.c_int32
        L.spc_symbolic_export_rows.argtypes = [vp, vp, vp]
        L.spc_symbolic_export_rows.restype = C.c_int32
        L.spc_symbolic_export_pairs.argtypes = [vp, vp, vp, vp, vp, vp]
        L.spc_symbolic_export_pairs.restype = C.c_int32
        L.spc_symbolic_export_tasks.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), vp, vp]
        L.spc_symbolic_export_tasks.restype = C.c_int32
        L.spc_symbolic_free.argtypes = [vp]
        L.spc_symbolic_free.restype = C.c_int32
        L.spc_factor.argtypes = [vp, vp, vp, C.POINTER(vp)]
        L.spc_factor.restype = C.c_int32
        L.spc_refactor.argtypes = [vp, vp, vp]
        L.spc_refactor.restype = C.c_int32
        L.spc_numeric_status.argtypes = [vp]
        L.spc_numeric_status.restype = C.c_int32
        L.spc_solve.argtypes = [vp, C.c_int32, vp, C.c_int64, vp, C.c_int64, vp]
        L.spc_solve.restype = C.c_int32
        L.spc_solve_noalloc.argtypes = [vp, C.c_int32, vp, C.c_int64, vp, C.c_int64, vp]
        L.spc_solve_noalloc.restype = C.c_int32
        L.spc_factor_export.argtypes = [vp, vp, vp, vp]
        L.spc_factor_export.restype = C.c_int32
        L.spc_numeric_free.argtypes = [vp]
        L.spc_numeric_free.restype = None
        L.spc_numeric_set_timing.argtypes = [vp, C.c_int32]
        L.spc_numeric_set_timing.restype = C.c_int32
        L.spc_numeric_get_timing.argtypes = [vp, C.POINTER(spc_kernel_times)]
        L.spc_numeric_get_timing.restype = C.c_int32
        L.spc_solve_refine.argtypes = [vp, C.c_int32, vp, C.c_int64, vp, C.c_int64, C.c_double,
                                       C.c_int32, vp, C.POINTER(C.c_int32), vp]
        L.spc_solve_refine.restype = C.c_int32
        L.spc_numeric_task_log.argtypes = [vp, C.POINTER(C.c_int64), vp, vp]
        L.spc_numeric_task_log.restype = C.c_int32
        L.spc_numeric_info_get.argtypes = [vp, C.POINTER(spc_numeric_info)]
        L.spc_numeric_info_get.restype = C.c_int32
        L.spc_server_default_options.argtypes = [C.POINTER(spc_server_options)]
        L.spc_server_default_options.restype = None
        L.spc_server_create.argtypes = [C.POINTER(spc_server_options), C.POINTER(vp)]
        L.spc_server_create.restype = C.c_int32
        L.spc_server_add_pattern.argtypes = [vp, vp, C.POINTER(C.c_int32)]
        L.spc_server_add_pattern.restype = C.c_int32
        L.spc_server_submit.argtypes = [vp, C.POINTER(spc_request), C.POINTER(C.c_int64)]
        L.spc_server_submit.restype = C.c_int32
        L.spc_server_wait.argtypes = [vp, C.c_int64, C.POINTER(spc_request_result)]
        L.spc_server_wait.restype = C.c_int32
        L.spc_server_stats_get.argtypes = [vp, C.POINTER(spc_server_stats)]
        L.spc_server_stats_get.restype = C.c_int32
        L.spc_server_destroy.argtypes = [vp]
        L.spc_server_destroy.restype = C.c_int32
        L.spc_measure_ceilings.argtypes = [C.POINTER(spc_ceilings)]
        L.spc_measure_ceilings.restype = C.c_int32
        L.spc_status_string.argtypes = [C.c_int32]
        L.spc_status_string.restype = C.c_char_p
        _lib = L
    return _lib


def status_string(st: int) -> str:
    return lib().spc_status_string(int(st)).decode()


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _stream_ptr(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


# ---------------------------------------------------------------------------
# symbolic
# ---------------------------------------------------------------------------

def _options(sn_cap=150, amalg_ratio=0.0, sched=0, mem_budget_bytes=0, spin_limit=0,
             debug_flags=0, precision=0, threads=0, small_w=0, small_r=0, deterministic=None,
             workers=0, solve_tail=0, upd_chunk=0):
    """spc_options; deterministic=None takes the library's default (1), except
    with sched 2, which needs 0."""
    opt = spc_options()
    lib().spc_default_options(C.byref(opt))
    opt.sn_cap = int(sn_cap)
    opt.sched = int(sched)
    opt.amalg_ratio = float(amalg_ratio)
    opt.mem_budget_bytes = int(mem_budget_bytes)
    opt.spin_limit = int(spin_limit)
    opt.debug_flags = int(debug_flags)
    opt.precision = int(precision)
    opt.threads = int(threads)
    opt.small_w = int(small_w)
    opt.small_r = int(small_r)
    if deterministic is not None:
        opt.deterministic = int(deterministic)
    elif int(sched) == 2:
        opt.deterministic = 0
    opt.workers = int(workers)
    opt.solve_tail = int(solve_tail)
    opt.upd_chunk = int(upd_chunk)
    return opt


class Symbolic:
    """spc_analyze: host symbolic analysis of the lower CSC pattern."""

    def __init__(self, n, colptr, rowind, perm=None, **opts):
        self.n = int(n)
        cp = _np(colptr, np.int64)
        ri = _np(rowind, np.int32)
        pm = None if perm is None else _np(perm, np.int32)
        opt = _options(**opts)
        h = C.c_void_p()
        if ri.size == 0:
            ri = np.zeros(1, dtype=np.int32)
        st = lib().spc_analyze(self.n, _ptr(cp), _ptr(ri), _ptr(pm), C.byref(opt), C.byref(h))
        if st != SPC_OK:
            raise SpcError(st, "spc_analyze")
        self.handle = h
        self.perm = np.arange(self.n, dtype=np.int32) if pm is None else pm.copy()
        self.batch_ptr = np.array([0, self.n], dtype=np.int64)

    @classmethod
    def batch(cls, mats, **opts):
        """spc_analyze_batch over mats = [(n, colptr, rowind, perm or None), ...]."""
        self = cls.__new__(cls)
        count = len(mats)
        ns = np.array([int(m[0]) for m in mats], dtype=np.int64)
        keep = []
        cps = (C.c_void_p * max(count, 1))()
        ris = (C.c_void_p * max(count, 1))()
        pms = (C.c_void_p * max(count, 1))()
        any_perm = False
        for k, m in enumerate(mats):
            cp = _np(m[1], np.int64)
            ri = _np(m[2], np.int32)
            if ri.size == 0:
                ri = np.zeros(1, dtype=np.int32)
            pm = None if len(m) < 4 or m[3] is None else _np(m[3], np.int32)
            keep += [cp, ri, pm]
            cps[k] = cp.ctypes.data
            ris[k] = ri.ctypes.data
            pms[k] = None if pm is None else pm.ctypes.data
            any_perm |= pm is not None
        opt = _options(**opts)
        h = C.c_void_p()
        st = lib().spc_analyze_batch(count, _ptr(ns) if count else None, cps, ris,
                                     pms if any_perm else None, C.byref(opt), C.byref(h))
        if st != SPC_OK:
            raise SpcError(st, "spc_analyze_batch")
        self.handle = h
        self.n = int(ns.sum())
        self.batch_ptr = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
        self.perm = None
        return self

    def info(self) -> dict:
        inf = spc_symbolic_info()
        st = lib().spc_symbolic_info_get(self.handle, C.byref(inf))
        if st != SPC_OK:
            raise SpcError(st, "spc_symbolic_info_get")
        return {f: getattr(inf, f) for f, _ in spc_symbolic_info._fields_}

    def export(self):
        inf = self.info()
        n, ns = inf["n"], inf["nsup"]
        parent = np.zeros(max(n, 1), dtype=np.int32)
        cc = np.zeros(max(n, 1), dtype=np.int32)
        sp = np.zeros(ns + 1, dtype=np.int32)
        spar = np.zeros(max(ns, 1), dtype=np.int32)
        st = lib().spc_symbolic_export(self.handle, _ptr(parent), _ptr(cc), _ptr(sp), _ptr(spar))
        if st != SPC_OK:
            raise SpcError(st, "spc_symbolic_export")
        return parent[:n], cc[:n], sp, spar[:ns]

    def rows(self):
        ns = self.info()["nsup"]
        rp = np.zeros(ns + 1, dtype=np.int64)
        lib().spc_symbolic_export_rows(self.handle, _ptr(rp), None)
        rows = np.zeros(max(int(rp[-1]), 1), dtype=np.int32)
        lib().spc_symbolic_export_rows(self.handle, None, _ptr(rows))
        return rp, rows[: int(rp[-1])]

    def pairs(self):
        inf = self.info()
        npairs, nrel = inf["npairs"], inf["nrel"]
        src = np.zeros(max(npairs, 1), dtype=np.int32)
        tgt = np.zeros(max(npairs, 1), dtype=np.int32)
        seg = np.zeros(max(2 * npairs, 2), dtype=np.int32)
        ro = np.zeros(max(npairs, 1), dtype=np.int64)
        rel = np.zeros(max(nrel, 1), dtype=np.int32)
        st = lib().spc_symbolic_export_pairs(self.handle, _ptr(src), _ptr(tgt), _ptr(seg), _ptr(ro),
                                             _ptr(rel))
        if st != SPC_OK:
            raise SpcError(st, "spc_symbolic_export_pairs")
        return dict(src=src[:npairs], tgt=tgt[:npairs], seg=seg[: 2 * npairs].reshape(-1, 2),
                    rel_off=ro[:npairs], rel=rel[:nrel])

    def tasks(self, workers=256):
        """Task order of the task-queue schedule: (tasks[ntasks, 4] as
        (kind, s, a, b), cnt0[nsup])."""
        nt = C.c_int64(0)
        st = lib().spc_symbolic_export_tasks(self.handle, int(workers), C.byref(nt), None, None)
        if st != SPC_OK:
            raise SpcError(st, "spc_symbolic_export_tasks")
        tk = np.zeros(max(4 * nt.value, 4), dtype=np.int32)
        cnt0 = np.zeros(max(self.info()["nsup"], 1), dtype=np.int32)
        st = lib().spc_symbolic_export_tasks(self.handle, int(workers), C.byref(nt), _ptr(tk),
                                             _ptr(cnt0))
        if st != SPC_OK:
            raise SpcError(st, "spc_symbolic_export_tasks")
        return tk[: 4 * nt.value].reshape(-1, 4), cnt0[: self.info()["nsup"]]

    def free(self):
        if getattr(self, "handle", None):
            st = lib().spc_symbolic_free(self.handle)
            if st != SPC_OK:
                raise SpcError(st, "spc_symbolic_free")
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().spc_symbolic_free(self.handle)
        except Exception:
            pass


# ---------------------------------------------------------------------------
# numeric
# ---------------------------------------------------------------------------

def _dev_f64(t, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("%s must be a float64 tensor on the GPU" % name)
    return t


class Numeric:
    """spc_factor: device numeric factorization; owns the factor's device memory."""

    def __init__(self, sym: Symbolic, values, stream=None):
        values = _dev_f64(values, "values").contiguous()
        self.sym = sym
        self._values = values  # keep alive until the stream has consumed it
        h = C.c_void_p()
        st = lib().spc_factor(sym.handle, C.c_void_p(values.data_ptr()), _stream_ptr(stream),
                              C.byref(h))
        if st != SPC_OK:
            raise SpcError(st, "spc_factor")
        self.handle = h

    def refactor(self, values, stream=None):
        values = _dev_f64(values, "values").contiguous()
        self._values = values
        st = lib().spc_refactor(self.handle, C.c_void_p(values.data_ptr()), _stream_ptr(stream))
        if st != SPC_OK:
            raise SpcError(st, "spc_refactor")

    def status(self) -> int:
        return int(lib().spc_numeric_status(self.handle))

    def _operands(self, b, x):
        """Column-major (n, k) views of b and x (x allocated when None)."""
        import torch

        b = _dev_f64(b, "b")
        n = self.sym.n
        one = b.dim() == 1
        B = b.reshape(n, 1) if one else b
        if B.shape[0] != n:
            raise ValueError("b has %d rows, expected %d" % (B.shape[0], n))
        k = B.shape[1]
        if B.stride(0) != 1 or (k > 1 and B.stride(1) < n):
            B = B.t().contiguous().t()  # column-major copy
        ldb = max(B.stride(1) if k > 1 else n, n)
        if x is None:
            X = torch.empty((k, n), dtype=torch.float64, device=b.device).t()
        else:
            X = _dev_f64(x, "x").reshape(n, k)
            if X.stride(0) != 1 or (k > 1 and X.stride(1) < n):
                raise ValueError("x must be column-major (n, k)")
        ldx = max(X.stride(1) if k > 1 else n, n)
        return one, B, ldb, X, ldx, k

    def solve(self, b, x=None, stream=None):
        """x = A^{-1} b; b is (n,) or (n, k); returns x with b's shape."""
        one, B, ldb, X, ldx, k = self._operands(b, x)
        st = lib().spc_solve(self.handle, k, C.c_void_p(B.data_ptr()), ldb,
                             C.c_void_p(X.data_ptr()), ldx, _stream_ptr(stream))
        if st != SPC_OK:
            raise SpcError(st, "spc_solve")
        return X.reshape(self.sym.n) if one else X

    def solve_noalloc(self, b, x, stream=None):
        """spc_solve_noalloc: x = A^{-1} b into the caller's x (no device
        allocation anywhere on the call's path, x included): b and x must be
        column-major (n,) or (n, k) GPU float64 tensors; nothing is copied."""
        n = self.sym.n
        one = b.dim() == 1
        B = _dev_f64(b, "b").reshape(n, -1)
        X = _dev_f64(x, "x").reshape(n, -1)
        k = B.shape[1]
        for t, nm in ((B, "b"), (X, "x")):
            if t.shape[1] != k or t.stride(0) != 1 or (k > 1 and t.stride(1) < n):
                raise ValueError("%s must be column-major (n, %d)" % (nm, k))
        ldb = max(B.stride(1) if k > 1 else n, n)
        ldx = max(X.stride(1) if k > 1 else n, n)
        st = lib().spc_solve_noalloc(self.handle, k, C.c_void_p(B.data_ptr()), ldb,
                                     C.c_void_p(X.data_ptr()), ldx, _stream_ptr(stream))
        if st != SPC_OK:
            raise SpcError(st, "spc_solve_noalloc")
        return X.reshape(self.sym.n) if one else X

    def solve_refine(self, b, x=None, tol=1e-10, max_iter=10, stream=None, check=True):
        """Iterative refinement in FP64 (spc_solve_refine).  Returns (x, iters,
        berr); raises SpcError unless converged when check is set."""
        one, B, ldb, X, ldx, k = self._operands(b, x)
        it = C.c_int32(0)
        berr = np.zeros(max(k * max(len(self.sym.batch_ptr) - 1, 1), 1), dtype=np.float64)
        st = lib().spc_solve_refine(self.handle, k, C.c_void_p(B.data_ptr()), ldb,
                                    C.c_void_p(X.data_ptr()), ldx, float(tol), int(max_iter),
                                    _stream_ptr(stream), C.byref(it), _ptr(berr))
        self.last_refine_status = int(st)
        if st != SPC_OK and (check or st != SPC_ERR_NOT_CONVERGED):
            raise SpcError(st, "spc_solve_refine")
        nb = len(self.sym.batch_ptr) - 1
        if nb > 1:  # (matrix, column) backward errors of a batch
            berr = berr[: k * nb].reshape(k, nb).T
        else:
            berr = berr[:k]
        return (X.reshape(self.sym.n) if one else X), int(it.value), berr

    def info(self) -> dict:
        t = spc_numeric_info()
        st = lib().spc_numeric_info_get(self.handle, C.byref(t))
        if st != SPC_OK:
            raise SpcError(st, "spc_numeric_info_get")
        return {f: getattr(t, f) for f, _ in t._fields_}

    def set_timing(self, enable=True):
        st = lib().spc_numeric_set_timing(self.handle, int(bool(enable)))
        if st != SPC_OK:
            raise SpcError(st, "spc_numeric_set_timing")

    def timing(self) -> dict:
        """Per-kernel-class device ms and launch counts of the last factorization."""
        t = spc_kernel_times()
        st = lib().spc_numeric_get_timing(self.handle, C.byref(t))
        if st != SPC_OK:
            raise SpcError(st, "spc_numeric_get_timing")
        out = {c: dict(ms=t.ms[i], launches=t.launches[i]) for i, c in enumerate(KERNEL_CLASSES)}
        out["total_ms"] = t.total_ms
        return out

    def task_log(self):
        """spc_numeric_task_log: (tasks[ntasks, 4], stamps[ntasks, 2])."""
        nt = C.c_int64(0)
        st = lib().spc_numeric_task_log(self.handle, C.byref(nt), None, None)
        if st != SPC_OK:
            raise SpcError(st, "spc_numeric_task_log")
        tk = np.zeros(max(4 * nt.value, 4), dtype=np.int32)
        sp = np.zeros(max(2 * nt.value, 2), dtype=np.int32)
        st = lib().spc_numeric_task_log(self.handle, C.byref(nt), _ptr(tk), _ptr(sp))
        if st != SPC_OK:
            raise SpcError(st, "spc_numeric_task_log")
        return tk[: 4 * nt.value].reshape(-1, 4), sp[: 2 * nt.value].reshape(-1, 2)

    def export(self):
        """Host copy (Sp, Si, Sx) of L in the stored supernodal column structure."""
        nnz = self.sym.info()["nnz_stored"]
        n = self.sym.n
        Sp = np.zeros(n + 1, dtype=np.int64)
        Si = np.zeros(max(nnz, 1), dtype=np.int32)
        Sx = np.zeros(max(nnz, 1), dtype=np.float64)
        st = lib().spc_factor_export(self.handle, _ptr(Sp), _ptr(Si), _ptr(Sx))
        if st != SPC_OK:
            raise SpcError(st, "spc_factor_export")
        return Sp, Si[:nnz], Sx[:nnz]

    def free(self):
        if getattr(self, "handle", None):
            lib().spc_numeric_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# request server
# ---------------------------------------------------------------------------

def request_operands(n, nnz_a, values, b, x):
    """Checks a server request's device operands: float64 tensors on the GPU,
    b and x column-major (n, k), values contiguous with nnz_a entries.
    Returns (values, B, X) with B and X as (n, k) views."""
    if values is not None:
        values = _dev_f64(values, "values").contiguous()
        if values.numel() != nnz_a:
            raise ValueError("values has %d entries, expected %d" % (values.numel(), nnz_a))
    B = _dev_f64(b, "b").reshape(n, -1)
    X = _dev_f64(x, "x").reshape(n, -1)
    if B.shape[1] != X.shape[1]:
        raise ValueError("b and x have different column counts")
    k = B.shape[1]
    for t, nm in ((B, "b"), (X, "x")):
        if t.stride(0) != 1 or (k > 1 and t.stride(1) < n):
            raise ValueError("%s must be column-major (n, k)" % nm)
    return values, B, X


class Server:
    """spc_server_*: continuous batching of factor+solve / solve-only requests."""

    def __init__(self, max_inflight=8, max_nrhs=64, mem_budget_bytes=0):
        opt = spc_server_options()
        lib().spc_server_default_options(C.byref(opt))
        opt.max_inflight = int(max_inflight)
        opt.max_nrhs = int(max_nrhs)
        opt.mem_budget_bytes = int(mem_budget_bytes)
        h = C.c_void_p()
        st = lib().spc_server_create(C.byref(opt), C.byref(h))
        if st != SPC_OK:
            raise SpcError(st, "spc_server_create")
        self.handle = h
        self._patterns = []
        self._keep = {}

    def add_pattern(self, sym: Symbolic) -> int:
        pid = C.c_int32(0)
        st = lib().spc_server_add_pattern(self.handle, sym.handle, C.byref(pid))
        if st != SPC_OK:
            raise SpcError(st, "spc_server_add_pattern")
        self._patterns.append(sym)
        return int(pid.value)

    def submit(self, pattern, b, x, values=None, kind=None, stream=None) -> int:
        """b, x: column-major (n, k) float64 device tensors (x written);
        values given: factor then solve (kind 0), else solve only (kind 1).
        The request runs after the work enqueued on `stream` (torch's current
        stream by default) up to this call."""
        sym = self._patterns[pattern]
        values, B, X = request_operands(sym.n, sym.info()["nnz_a"], values, b, x)
        r = spc_request()
        r.pattern = int(pattern)
        r.kind = int((0 if values is not None else 1) if kind is None else kind)
        n = sym.n
        k = B.shape[1]
        r.nrhs = k
        r.values = None if values is None else values.data_ptr()
        r.b, r.ldb = B.data_ptr(), max(B.stride(1) if k > 1 else n, n)
        r.x, r.ldx = X.data_ptr(), max(X.stride(1) if k > 1 else n, n)
        r.stream = _stream_ptr(stream)
        t = C.c_int64(0)
        st = lib().spc_server_submit(self.handle, C.byref(r), C.byref(t))
        if st != SPC_OK:
            raise SpcError(st, "spc_server_submit")
        self._keep[int(t.value)] = (values, B, X, b, x)
        return int(t.value)

    def wait(self, ticket) -> dict:
        res = spc_request_result()
        st = lib().spc_server_wait(self.handle, int(ticket), C.byref(res))
        if st != SPC_OK:
            raise SpcError(st, "spc_server_wait")
        self._keep.pop(int(ticket), None)
        return {"status": res.status, "queue_ms": res.queue_ms, "latency_ms": res.latency_ms}

    def stats(self) -> dict:
        t = spc_server_stats()
        st = lib().spc_server_stats_get(self.handle, C.byref(t))
        if st != SPC_OK:
            raise SpcError(st, "spc_server_stats_get")
        return {f: getattr(t, f) for f, _ in t._fields_}

    def destroy(self):
        if getattr(self, "handle", None):
            lib().spc_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def measure_ceilings() -> dict:
    """spc_measure_ceilings: measured FP64/FP32 matrix-core TFLOP/s and copy GB/s."""
    c = spc_ceilings()
    st = lib().spc_measure_ceilings(C.byref(c))
    if st != SPC_OK:
        raise SpcError(st, "spc_measure_ceilings")
    return {f: getattr(c, f) for f, _ in c._fields_}


# C-ABI-named entry points
def analyze(n, colptr, rowind, perm=None, **opts) -> Symbolic:
    return Symbolic(n, colptr, rowind, perm, **opts)


def analyze_batch(mats, **opts) -> Symbolic:
    return Symbolic.batch(mats, **opts)


def factor(sym: Symbolic, values, stream=None) -> Numeric:
    return Numeric(sym, values, stream)


def refactor(num: Numeric, values, stream=None) -> None:
    num.refactor(values, stream)


def numeric_status(num: Numeric) -> int:
    return num.status()


def solve(num: Numeric, b, x=None, stream=None):
    return num.solve(b, x, stream)


def solve_noalloc(num: Numeric, b, x, stream=None):
    return num.solve_noalloc(b, x, stream)


def solve_refine(num: Numeric, b, x=None, tol=1e-10, max_iter=10, stream=None):
    return num.solve_refine(b, x, tol, max_iter, stream)


def numeric_info_get(num: Numeric) -> dict:
    return num.info()


def factor_export(num: Numeric):
    return num.export()


def symbolic_free(sym: Symbolic) -> None:
    sym.free()


def numeric_free(num: Numeric) -> None:
    num.free()

