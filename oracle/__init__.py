"""CPU oracle for the supernodal Cholesky path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline legs of
``bench.py`` (``cpu_baseline``; ``cpu_batch_baseline``, whose pool workers run
this package) may import this package.  It wraps ``oracle.c`` (plain C, one
core, IEEE binary64, built with ``-O2 -ffp-contract=off``) through ctypes and
shares no code with the HIP library.

Functions and the paper passages they follow (arXiv:1608.00044):

* ``permute``       -- C = lower(P A P^T), the ordering applied before factoring (Section V).
* ``symbolic``      -- fill, elimination tree and column counts by their
                       definitions (Section II-B).
* ``supernodes``    -- non-fundamental supernodes (Section II-B) with the
                       150-column cap split (Section III-B).
* ``amalgamate``    -- relaxed amalgamation; the paper is silent, the rule is
                       the documented reading.  Parity unpinned by the paper:
                       pinned only by the stated rule and its invariants.
* ``factor``        -- left-looking column Cholesky, Algorithm 1 reorganised as
                       in Section II-C.
* ``solve``         -- the two triangular solves (Section II-A).
* ``residual_exact``, ``residual_probe``, ``backward_error`` -- checks.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
F64P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _opt(p):
    return None if p is None else p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        L.orc_validate.argtypes = [C.c_int64, vp, vp, vp]
        L.orc_validate.restype = C.c_int
        L.orc_permute.argtypes = [C.c_int64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_permute.restype = C.c_int
        L.orc_sym_new.argtypes = [C.c_int64, vp, vp]
        L.orc_sym_new.restype = vp
        L.orc_sym_nnz.argtypes = [vp]
        L.orc_sym_nnz.restype = C.c_int64
        L.orc_sym_get.argtypes = [vp, vp, vp, vp, vp]
        L.orc_sym_get.restype = None
        L.orc_sym_free.argtypes = [vp]
        L.orc_sym_free.restype = None
        L.orc_supernodes.argtypes = [C.c_int64, vp, vp, C.c_int32, vp]
        L.orc_supernodes.restype = C.c_int64
        L.orc_amalgamate.argtypes = [C.c_int64, vp, vp, C.c_int64, vp, C.c_int32, C.c_double]
        L.orc_amalgamate.restype = C.c_int64
        L.orc_factor.argtypes = [C.c_int64, vp, vp, vp, vp, vp, vp]
        L.orc_factor.restype = C.c_int
        L.orc_solve.argtypes = [C.c_int64, vp, vp, vp, vp, C.c_int64, vp, C.c_int64, vp,
                                C.c_int64]
        L.orc_solve.restype = C.c_int
        L.orc_symv.argtypes = [C.c_int64, vp, vp, vp, C.c_int64, vp, C.c_int64, vp, C.c_int64]
        L.orc_symv.restype = None
        L.orc_residual_exact.argtypes = [C.c_int64, vp, vp, vp, vp, vp, vp]
        L.orc_residual_exact.restype = C.c_double
        L.orc_residual_probe.argtypes = [C.c_int64, vp, vp, vp, vp, vp, vp, C.c_int64, vp]
        L.orc_residual_probe.restype = C.c_double
        L.orc_backward_error.argtypes = [C.c_int64, vp, vp, vp, C.c_int64, vp, C.c_int64, vp,
                                         C.c_int64, vp]
        L.orc_backward_error.restype = None
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def validate(n, colptr, rowind, perm=None) -> int:
    cp, ri = _i64(colptr), _i32(rowind)
    pm = None if perm is None else _i32(perm)
    return lib().orc_validate(n, _p(cp), _p(ri), _p(pm))


def permute(n, colptr, rowind, values=None, perm=None):
    """Return (Cp, Ci, Cx, map) of C = lower(P A P^T)."""
    cp, ri = _i64(colptr), _i32(rowind)
    vx = None if values is None else _f64(values)
    pm = None if perm is None else _i32(perm)
    nnz = int(cp[n]) if n else 0
    Cp = np.zeros(n + 1, dtype=np.int64)
    Ci = np.zeros(max(nnz, 1), dtype=np.int32)
    Cx = np.zeros(max(nnz, 1), dtype=np.float64)
    mp = np.zeros(max(nnz, 1), dtype=np.int64)
    st = lib().orc_permute(n, _p(cp), _p(ri), _p(vx), _p(pm), _p(Cp), _p(Ci), _p(Cx), _p(mp))
    if st:
        raise OracleError("permute failed: %d" % st)
    return Cp, Ci[:nnz], Cx[:nnz], mp[:nnz]


@dataclass
class Symbolic:
    n: int
    parent: np.ndarray
    colcount: np.ndarray
    Lp: np.ndarray
    Li: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.Lp[-1])

    @property
    def flops(self) -> int:
        """Algorithmic flop count sum_j colcount(j)^2 (exact structure)."""
        c = self.colcount.astype(np.int64)
        return int(np.sum(c * c))


def symbolic(n, Cp, Ci) -> Symbolic:
    Cp, Ci = _i64(Cp), _i32(Ci)
    h = lib().orc_sym_new(n, _p(Cp), _p(Ci))
    if not h:
        raise OracleError("symbolic analysis failed")
    try:
        nnz = lib().orc_sym_nnz(h)
        parent = np.zeros(n, dtype=np.int32)
        cc = np.zeros(n, dtype=np.int32)
        Lp = np.zeros(n + 1, dtype=np.int64)
        Li = np.zeros(max(nnz, 1), dtype=np.int32)
        lib().orc_sym_get(h, _p(parent), _p(cc), _p(Lp), _p(Li))
    finally:
        lib().orc_sym_free(h)
    return Symbolic(n, parent, cc, Lp, Li[:nnz])


def supernodes(n, parent, colcount, cap=150) -> np.ndarray:
    parent, cc = _i32(parent), _i32(colcount)
    sp = np.zeros(n + 1, dtype=np.int32)
    ns = lib().orc_supernodes(n, _p(parent), _p(cc), cap, _p(sp))
    if ns < 0:
        raise OracleError("supernodes failed: %d" % ns)
    return sp[: ns + 1].copy()


def amalgamate(n, parent, colcount, sn_ptr, cap=150, ratio=0.1) -> np.ndarray:
    parent, cc = _i32(parent), _i32(colcount)
    sp = _i32(sn_ptr).copy()
    ns = lib().orc_amalgamate(n, _p(parent), _p(cc), len(sp) - 1, _p(sp), cap, ratio)
    if ns < 0:
        raise OracleError("amalgamate failed: %d" % ns)
    return sp[: ns + 1].copy()


def supernode_partition(n, parent, colcount, cap=150, ratio=0.0) -> np.ndarray:
    sp = supernodes(n, parent, colcount, cap)
    if ratio > 0.0:
        sp = amalgamate(n, parent, colcount, sp, cap, ratio)
    return sp


def supernodal_parent(parent, sn_ptr) -> np.ndarray:
    """Supernodal elimination tree: the supernode holding parent(last column)."""
    n = len(parent)
    owner = np.zeros(n, dtype=np.int64)
    for s in range(len(sn_ptr) - 1):
        owner[sn_ptr[s]:sn_ptr[s + 1]] = s
    out = np.full(len(sn_ptr) - 1, -1, dtype=np.int32)
    for s in range(len(sn_ptr) - 1):
        p = parent[sn_ptr[s + 1] - 1]
        out[s] = -1 if p < 0 else owner[p]
    return out


def factor(n, Cp, Ci, Cx, sym: Symbolic):
    """Return (status, Lx) with Lx aligned to sym.Li."""
    Cp, Ci, Cx = _i64(Cp), _i32(Ci), _f64(Cx)
    Lx = np.zeros(max(sym.nnz, 1))
    st = lib().orc_factor(n, _p(Cp), _p(Ci), _p(Cx), _p(sym.Lp), _p(sym.Li), _p(Lx))
    if st < 0:
        raise OracleError("factor failed: %d" % st)
    return st, Lx[: sym.nnz]


def solve(n, sym: Symbolic, Lx, perm, b):
    b = np.asarray(b, dtype=np.float64)
    one = b.ndim == 1
    B = np.ascontiguousarray(b.reshape(n, -1).T)  # column c contiguous
    nrhs = B.shape[0]
    X = np.zeros_like(B)
    pm = None if perm is None else _i32(perm)
    st = lib().orc_solve(n, _p(sym.Lp), _p(sym.Li), _p(_f64(Lx)), _p(pm), nrhs, _p(B), n,
                         _p(X), n)
    if st:
        raise OracleError("solve failed: %d" % st)
    X = X.T
    return X[:, 0].copy() if one else np.asfortranarray(X)


def symv(n, colptr, rowind, values, z):
    z = np.asarray(z, dtype=np.float64)
    one = z.ndim == 1
    Z = np.ascontiguousarray(z.reshape(n, -1).T)
    Y = np.zeros_like(Z)
    lib().orc_symv(n, _p(_i64(colptr)), _p(_i32(rowind)), _p(_f64(values)), Z.shape[0],
                   _p(Z), n, _p(Y), n)
    Y = Y.T
    return Y[:, 0].copy() if one else Y


def residual_exact(n, Cp, Ci, Cx, sym: Symbolic, Lx) -> float:
    return lib().orc_residual_exact(n, _p(_i64(Cp)), _p(_i32(Ci)), _p(_f64(Cx)), _p(sym.Lp),
                                    _p(sym.Li), _p(_f64(Lx)))


def residual_probe(n, Cp, Ci, Cx, sym: Symbolic, Lx, Z) -> float:
    Z = np.ascontiguousarray(np.asarray(Z, dtype=np.float64).reshape(n, -1).T)
    return lib().orc_residual_probe(n, _p(_i64(Cp)), _p(_i32(Ci)), _p(_f64(Cx)), _p(sym.Lp),
                                    _p(sym.Li), _p(_f64(Lx)), Z.shape[0], _p(Z))


def backward_error(n, colptr, rowind, values, b, x):
    b = np.asarray(b, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    B = np.ascontiguousarray(b.reshape(n, -1).T)
    X = np.ascontiguousarray(x.reshape(n, -1).T)
    eta = np.zeros(B.shape[0])
    lib().orc_backward_error(n, _p(_i64(colptr)), _p(_i32(rowind)), _p(_f64(values)),
                             B.shape[0], _p(B), n, _p(X), n, _p(eta))
    return eta


def run(problem, cap=150, ratio=0.0, want_solve=True):
    """Whole oracle pipeline on an ``inputs.Problem``: permute, symbolic,
    supernode partition, factor and (optionally) solve."""
    n = problem.n
    Cp, Ci, Cx, _ = permute(n, problem.colptr, problem.rowind, problem.values, problem.perm)
    sym = symbolic(n, Cp, Ci)
    sn = supernode_partition(n, sym.parent, sym.colcount, cap, ratio)
    st, Lx = factor(n, Cp, Ci, Cx, sym)
    out = dict(C=(Cp, Ci, Cx), sym=sym, sn_ptr=sn, status=st, Lx=Lx)
    if want_solve and st == 0 and problem.rhs is not None:
        out["x"] = solve(n, sym, Lx, problem.perm, problem.rhs)
    return out
