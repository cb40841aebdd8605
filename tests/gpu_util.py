"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare it with the oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from paper_1608_00044_amd import spchol


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch


def gpu_factor(p, cap=150, ratio=0.0, sched=0, deterministic=None, **opts):
    """Analyze + factor on cuda:0; returns (sym, num, values_tensor).
    deterministic=None: the library's default order (sched 2: atomic)."""
    torch = torch_dev()
    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=cap, amalg_ratio=ratio,
                         sched=sched, deterministic=deterministic, **opts)
    vals = torch.from_numpy(np.ascontiguousarray(p.values)).to("cuda:0")
    num = spchol.factor(sym, vals)
    return sym, num, vals


def exact_values(num, osym):
    """GPU factor values on the oracle's exact structure, plus the values the
    GPU stores outside it (must be explicit zeros)."""
    Sp, Si, Sx = num.export()
    n = osym.n
    cols_s = np.repeat(np.arange(n, dtype=np.int64), np.diff(Sp))
    keys_s = cols_s * n + Si
    cols_o = np.repeat(np.arange(n, dtype=np.int64), np.diff(osym.Lp))
    keys_o = cols_o * n + osym.Li
    pos = np.searchsorted(keys_s, keys_o)
    assert (pos < keys_s.size).all() and np.array_equal(keys_s[pos], keys_o), \
        "stored structure does not contain the exact structure"
    extra = np.ones(keys_s.size, dtype=bool)
    extra[pos] = False
    return Sx[pos], Sx[extra]


def entry_tolerance(osym, Lx_ref, Cp, Ci, Cx):
    """|dL_ij| <= 1e-10 |L_ij| + 1e-13 sqrt(c_ii c_jj) / L_jj (c = diag of P A P^T)."""
    n = osym.n
    diag = np.zeros(n)
    nz = Cp[1:] > Cp[:-1]
    idx = Cp[:-1][nz]
    js = np.arange(n)[nz]
    isdiag = Ci[idx] == js
    diag[js[isdiag]] = Cx[idx[isdiag]]
    cols = np.repeat(np.arange(n), np.diff(osym.Lp))
    rows = osym.Li
    ljj = Lx_ref[osym.Lp[:-1]][cols]
    floor = 1e-13 * np.sqrt(np.abs(diag[rows] * diag[cols])) / np.abs(ljj)
    return 1e-10 * np.abs(Lx_ref) + floor


def compare_factor(p, num, cap=150, ratio=0.0, label=""):
    """Element-by-element parity of the GPU factor with the oracle's; returns
    (max violation ratio, residual of the GPU factor)."""
    Cp, Ci, Cx, _ = oracle.permute(p.n, p.colptr, p.rowind, p.values, p.perm)
    osym = oracle.symbolic(p.n, Cp, Ci)
    st, Lx = oracle.factor(p.n, Cp, Ci, Cx, osym)
    assert st == 0, "oracle failed on %s" % label
    got, extra = exact_values(num, osym)
    assert (extra == 0.0).all(), "explicit zeros of the amalgamated storage are not zero"
    tol = entry_tolerance(osym, Lx, Cp, Ci, Cx)
    err = np.abs(got - Lx)
    worst = float((err / tol).max()) if err.size else 0.0
    rho = oracle.residual_exact(p.n, Cp, Ci, Cx, osym, got)
    return worst, rho, (osym, Lx, got)


def eta_agreement_atol(p):
    """Bound on |eta_lib - eta_oracle| for one solution: both evaluate
    r = b - A x in FP64, each within gamma_m (|A||x| + |b|) per row (m = the
    row's entries + 1, Higham's dot-product bound), so the normwise backward
    errors differ by at most about 2 gamma_m <= 2.1 m u absolutely; twice
    that, with m the largest row of the full symmetric A."""
    col = np.repeat(np.arange(p.n), np.diff(p.colptr))
    off = p.rowind != col
    m = np.bincount(col, minlength=p.n) + np.bincount(p.rowind[off], minlength=p.n)
    return 4.2 * (int(m.max()) + 1) * np.finfo(np.float64).eps / 2
