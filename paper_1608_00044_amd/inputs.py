"""Seeded synthetic SPD inputs and the geometric nested-dissection ordering.

This module is input generation only: it builds the lower triangle of an SPD
matrix A in CSC form, a fill-reducing permutation for it and right-hand sides.
It contains none of the factorization's arithmetic and imports nothing from the
rest of the package, so the CPU oracle and the HIP path both consume exactly
the same arrays.

The paper orders its matrices with nested dissection (Section V, the Scotch
ordering paragraph) and evaluates on 3D finite-element, shell and circuit
matrices (Table I).  Those matrices are not available here; the stencil
matrices below stand in for them:

* 2D 5-point and 3D 7-point graph Laplacians (weights unit or lognormal) plus a
  diagonal shift: diag = sum of incident edge weights + shift.
* 3D 27-point stencil with 3 unknowns per node: each edge couples its two nodes
  through -W_e with W_e = G G^T / 3 (G a 3x3 matrix of N(0,1) draws) and each
  diagonal block is sum_e W_e + shift * I_3.

Conventions shared by every generator:
* nodes are numbered x fastest: id = x + kx * (y + ky * z);
* edges are enumerated node by node in increasing id, and for each node its
  forward neighbours in a fixed order; all random draws come from
  ``numpy.random.Generator(PCG64(seed))`` in that edge order, and right-hand
  sides are drawn from the same stream after the matrix;
* the returned CSC holds the lower triangle of the *unpermuted* A with the
  diagonal, rows sorted within each column, 0-based; ``perm[new] = old``.
"""
from __future__ import annotations

import functools
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """Lower-triangular CSC of an SPD matrix plus ordering and right-hand sides."""

    n: int
    colptr: np.ndarray  # int64[n+1]
    rowind: np.ndarray  # int32[nnz]
    values: np.ndarray  # float64[nnz]
    perm: np.ndarray | None  # int32[n], perm[new] = old; None = identity
    rhs: np.ndarray | None = None  # float64[n, nrhs], Fortran order
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])


# ---------------------------------------------------------------------------
# assembly helpers
# ---------------------------------------------------------------------------

def lower_csc_from_coo(n: int, rows, cols, vals):
    """Sum duplicate (row, col) entries and return the lower CSC (rows >= cols)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    if rows.size and np.any(rows < cols):
        raise ValueError("lower_csc_from_coo expects row >= col for every entry")
    key = cols * n + rows
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start) if vals.size else vals
    c = (uniq // n).astype(np.int64)
    r = (uniq % n).astype(np.int32)
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, c + 1, 1)
    colptr = np.cumsum(colptr)
    return colptr, r, summed


def lower_csc_from_dense(a: np.ndarray):
    """Lower CSC of the nonzero entries of a dense symmetric matrix (the
    diagonal is always stored)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    i, j = np.nonzero(np.tril(a != 0) | np.eye(n, dtype=bool))
    return lower_csc_from_coo(n, i, j, a[i, j])


def dense_from_lower_csc(n, colptr, rowind, values, perm=None):
    """Dense symmetric matrix from its lower CSC; with perm, returns P A P^T
    where (P A P^T)[i, j] = A[perm[i], perm[j]]."""
    a = np.zeros((n, n))
    for j in range(n):
        for p in range(colptr[j], colptr[j + 1]):
            i = rowind[p]
            a[i, j] += values[p]
            if i != j:
                a[j, i] += values[p]
    if perm is not None:
        perm = np.asarray(perm)
        a = a[np.ix_(perm, perm)]
    return a


# ---------------------------------------------------------------------------
# geometric nested dissection
# ---------------------------------------------------------------------------

def _box_ids(lo, hi, dims):
    """Node ids of the box [lo, hi) in natural order (x fastest)."""
    ndim = len(dims)
    if any(hi[d] <= lo[d] for d in range(ndim)):
        return np.zeros(0, dtype=np.int64)
    ids = np.zeros([1] * ndim, dtype=np.int64)
    stride = 1
    for d in range(ndim):
        shape = [1] * ndim
        shape[ndim - 1 - d] = hi[d] - lo[d]  # slowest axis first
        ids = ids + (np.arange(lo[d], hi[d], dtype=np.int64) * stride).reshape(shape)
        stride *= dims[d]
    return ids.ravel()


@functools.lru_cache(maxsize=256)
def nested_dissection(dims: tuple) -> np.ndarray:
    """Geometric nested-dissection elimination order of a regular grid.

    Recursively split the box across its longest extent (ties go to the lowest
    axis, x < y < z) with a one-node-thick plane at lo + ext // 2; number the
    lower box, then the upper box, then the plane in natural order.  A single
    node is numbered as is.  Returns ``order`` with order[new] = old node id.
    """
    dims = tuple(int(d) for d in dims)
    ndim = len(dims)
    strides = [int(np.prod(dims[:d])) for d in range(ndim)]
    order = np.empty(int(np.prod(dims)), dtype=np.int64)
    pos = [0]

    def emit(lo, hi):
        if all(hi[d] - lo[d] == 1 for d in range(ndim)):
            order[pos[0]] = sum(lo[d] * strides[d] for d in range(ndim))
            pos[0] += 1
        else:
            ids = _box_ids(lo, hi, dims)
            order[pos[0]:pos[0] + ids.size] = ids
            pos[0] += ids.size

    def rec(lo, hi):
        ext = [hi[d] - lo[d] for d in range(ndim)]
        if min(ext) <= 0:
            return
        big = max(ext)
        if big == 1:
            emit(lo, hi)
            return
        ax = ext.index(big)
        mid = lo[ax] + big // 2
        lo_l, hi_l = list(lo), list(hi)
        hi_l[ax] = mid
        lo_r, hi_r = list(lo), list(hi)
        lo_r[ax] = mid + 1
        lo_s, hi_s = list(lo), list(hi)
        lo_s[ax], hi_s[ax] = mid, mid + 1
        rec(lo_l, hi_l)
        rec(lo_r, hi_r)
        emit(lo_s, hi_s)

    rec([0] * ndim, list(dims))
    assert pos[0] == order.size
    order.setflags(write=False)
    return order


def expand_dofs(order: np.ndarray, dof: int) -> np.ndarray:
    """Node order -> unknown order when each node carries ``dof`` consecutive unknowns."""
    if dof == 1:
        return np.asarray(order, dtype=np.int64)
    return (np.asarray(order, dtype=np.int64)[:, None] * dof + np.arange(dof)).ravel()


# ---------------------------------------------------------------------------
# stencil generators
# ---------------------------------------------------------------------------

def _forward_offsets(ndim: int, full: bool):
    """Forward neighbour offsets (neighbour id > node id), in a fixed order.

    full=False: the axis neighbours +x, +y (, +z).  full=True: every offset in
    {-1,0,1}^ndim that is lexicographically positive in (dz, dy, dx)."""
    if not full:
        offs = []
        for d in range(ndim):
            o = [0] * ndim
            o[d] = 1
            offs.append(tuple(o))
        return offs
    offs = []
    import itertools

    for rev in itertools.product((-1, 0, 1), repeat=ndim):
        # rev = (dz, dy, dx) or (dy, dx); positive in lexicographic order
        if rev > tuple([0] * ndim):
            offs.append(tuple(reversed(rev)))  # back to (dx, dy, dz)
    return offs


def _grid_edges(dims, full):
    """(u, v) pairs with v > u for the stencil, enumerated node by node in
    increasing u and, per node, in the forward-offset order."""
    ndim = len(dims)
    n = int(np.prod(dims))
    ids = np.arange(n, dtype=np.int64)
    coords = []
    rem = ids.copy()
    for d in range(ndim):
        coords.append(rem % dims[d])
        rem //= dims[d]
    strides = np.cumprod([1] + list(dims[:-1]))
    us, vs, ks = [], [], []
    for k, off in enumerate(_forward_offsets(ndim, full)):
        ok = np.ones(n, dtype=bool)
        delta = 0
        for d in range(ndim):
            c = coords[d] + off[d]
            ok &= (c >= 0) & (c < dims[d])
            delta += off[d] * strides[d]
        u = ids[ok]
        us.append(u)
        vs.append(u + delta)
        ks.append(np.full(u.size, k, dtype=np.int64))
    u = np.concatenate(us)
    v = np.concatenate(vs)
    k = np.concatenate(ks)
    order = np.lexsort((k, u))  # by node, then by offset rank
    return u[order], v[order]


@functools.lru_cache(maxsize=256)
def _laplacian_pattern(dims):
    """Edges and lower CSC pattern of the grid Laplacian, with the position
    in the CSC of every COO entry [(v, u) per edge, then the diagonal]."""
    n = int(np.prod(dims))
    u, v = _grid_edges(dims, full=False)
    rows = np.concatenate([v, np.arange(n)])
    cols = np.concatenate([u, np.arange(n)])
    order = np.argsort(cols * n + rows, kind="stable")  # the entries are distinct
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr)
    for a in (u, v, order, colptr):
        a.setflags(write=False)
    return n, u, v, colptr, rows[order].astype(np.int32), order


def grid_laplacian(dims, rng, sigma=None, shift=0.0):
    """Graph Laplacian of the 2D 5-point / 3D 7-point grid plus shift*I.

    Edge weights are 1 (sigma None) or lognormal(0, sigma) drawn in edge order;
    off-diagonal entries are -w and diag = sum of incident w + shift."""
    dims = tuple(int(d) for d in dims)
    n, u, v, colptr, rowind, order = _laplacian_pattern(dims)
    if sigma is None:
        w = np.ones(u.size)
    else:
        w = rng.lognormal(mean=0.0, sigma=sigma, size=u.size)
    # incident weights summed in edge order, first as u then as v
    deg = np.bincount(np.concatenate([u, v]), weights=np.concatenate([w, w]), minlength=n)
    vals = np.concatenate([-w, deg + shift])[order]
    return n, colptr.copy(), rowind.copy(), vals


def grid27_3dof(dims, rng, shift=1e-3):
    """3D 27-point stencil with 3 unknowns per node and Wishart edge blocks.

    For each edge e (in edge order) G_e is a 3x3 block of N(0,1) draws
    (row-major), W_e = G_e G_e^T / 3; A_uv = -W_e and A_uu = sum_e W_e + shift*I."""
    dims = tuple(int(d) for d in dims)
    nn = int(np.prod(dims))
    n = 3 * nn
    u, v = _grid_edges(dims, full=True)
    g = rng.standard_normal((u.size, 3, 3))
    w = np.einsum("eik,ejk->eij", g, g) / 3.0
    dblk = np.zeros((nn, 3, 3))
    np.add.at(dblk, u, w)
    np.add.at(dblk, v, w)
    dblk += shift * np.eye(3)
    a, b = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")  # a=row dof, b=col dof
    # off-diagonal blocks: row node v > col node u, all 9 entries
    r_off = (3 * v[:, None, None] + a).ravel()
    c_off = (3 * u[:, None, None] + b).ravel()
    x_off = (-w).ravel()
    # diagonal blocks: lower triangle only
    low = a >= b
    node = np.arange(nn)
    r_d = (3 * node[:, None, None] + a)[:, low].ravel()
    c_d = (3 * node[:, None, None] + b)[:, low].ravel()
    x_d = dblk[:, low].ravel()
    rows = np.concatenate([r_off, r_d])
    cols = np.concatenate([c_off, c_d])
    vals = np.concatenate([x_off, x_d])
    return (n,) + lower_csc_from_coo(n, rows, cols, vals)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

WORKLOADS = {
    # 2D 5-point Laplacian on 64x64, unit weights, +1e-3 shift, ND, 1 RHS
    "lap2d_5pt_64": dict(kind="lap", dims=(64, 64), sigma=None, shift=1e-3, nrhs=1,
                         amalg=0.0, cfg=1),
    # 3D 7-point Laplacian on 64^3, lognormal(0,1) weights, +1e-6, ND, amalgamation 0.1
    "lap3d_7pt_64": dict(kind="lap", dims=(64, 64, 64), sigma=1.0, shift=1e-6, nrhs=1,
                         amalg=0.1, cfg=2),
    # 3D 27-point, 3 dof, Wishart blocks, +1e-3, ND, 8 RHS
    "elast27_48": dict(kind="27pt3", dims=(48, 48, 48), shift=1e-3, nrhs=8, amalg=0.1, cfg=3),
}


def make_grid_problem(kind, dims, seed, sigma=None, shift=1e-3, nrhs=1, order=True):
    """Build a stencil problem with geometric-ND ordering and N(0,1) RHS."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = tuple(int(d) for d in dims)
    if kind == "lap":
        n, cp, ri, vx = grid_laplacian(dims, rng, sigma=sigma, shift=shift)
        dof = 1
    elif kind == "27pt3":
        n, cp, ri, vx = grid27_3dof(dims, rng, shift=shift)
        dof = 3
    else:
        raise ValueError(kind)
    perm = expand_dofs(nested_dissection(dims), dof).astype(np.int32) if order else None
    rhs = np.asfortranarray(rng.standard_normal((n, nrhs))) if nrhs else None
    return Problem(n, cp, ri.astype(np.int32), vx, perm, rhs,
                   meta=dict(kind=kind, dims=dims, seed=seed, sigma=sigma, shift=shift))


def make_workload(name, repeat=0, nrhs=None, dims=None):
    """Named workload; seed = 1000 * cfg + repeat.  ``dims`` overrides the grid
    (a smaller grid of the same recipe, used for bounded samples)."""
    w = WORKLOADS[name]
    seed = 1000 * w["cfg"] + repeat
    p = make_grid_problem(w["kind"], dims or w["dims"], seed, sigma=w.get("sigma"),
                          shift=w["shift"], nrhs=w["nrhs"] if nrhs is None else nrhs)
    p.meta.update(name=name, amalg=w["amalg"])
    return p


# Batch of independent 2D 5-point Laplacians: grid side uniform in
# [side_lo, side_hi], lognormal(0, 0.5) edge weights, diagonal = incident
# weight sum + shift, geometric nested dissection, one N(0, 1) right-hand side.
BATCH_RECIPE = dict(count=2000, side_lo=16, side_hi=128, sigma=0.5, shift=1e-3, nrhs=1, cfg=4)


def make_batch(count=None, seed=4000, side_lo=None, side_hi=None, nrhs=None, members=None):
    """List of Problems following BATCH_RECIPE (overrides shrink it for tests).
    `members` (indices into the batch) builds only those matrices, each the
    same as in the whole batch."""
    r = BATCH_RECIPE
    count = r["count"] if count is None else count
    lo = r["side_lo"] if side_lo is None else side_lo
    hi = r["side_hi"] if side_hi is None else side_hi
    nrhs = r["nrhs"] if nrhs is None else nrhs
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.integers(lo, hi + 1, size=count)
    ks = range(count) if members is None else members
    return [make_grid_problem("lap", (int(sides[k]), int(sides[k])), seed + 1 + k,
                              sigma=r["sigma"], shift=r["shift"], nrhs=nrhs) for k in ks]


def stack_batch(probs):
    """Concatenated values and right-hand sides of a batch (matrix k's rows
    after matrix k-1's), as the batched C ABI takes them."""
    vals = np.concatenate([p.values for p in probs]) if probs else np.zeros(0)
    rhs = None
    if probs and probs[0].rhs is not None:
        rhs = np.asfortranarray(np.concatenate([p.rhs for p in probs], axis=0))
    return vals, rhs


def block_diagonal(probs):
    """The direct sum of a batch as one Problem (the matrix a batched analysis
    factors), with the members' orderings and right-hand sides stacked."""
    n = sum(p.n for p in probs)
    cps, ris, pms = [np.zeros(1, dtype=np.int64)], [], []
    off, ent = 0, 0
    for p in probs:
        cps.append(np.asarray(p.colptr[1:], dtype=np.int64) + ent)
        ris.append(np.asarray(p.rowind, dtype=np.int64) + off)
        pm = np.arange(p.n) if p.perm is None else np.asarray(p.perm)
        pms.append(pm + off)
        off += p.n
        ent += int(p.colptr[-1])
    vals, rhs = stack_batch(probs)
    ri = np.concatenate(ris).astype(np.int32) if ris else np.zeros(0, dtype=np.int32)
    pm = np.concatenate(pms).astype(np.int32) if pms else np.zeros(0, dtype=np.int32)
    return Problem(n, np.concatenate(cps), ri, vals, pm, rhs)


# ---------------------------------------------------------------------------
# tiny cases
# ---------------------------------------------------------------------------

def tridiag(n, diag=2.0, off=-1.0):
    """tridiag(off, diag, off) in natural order (identity permutation)."""
    rows = np.concatenate([np.arange(n), np.arange(1, n)])
    cols = np.concatenate([np.arange(n), np.arange(n - 1)])
    vals = np.concatenate([np.full(n, diag), np.full(max(n - 1, 0), off)])
    cp, ri, vx = lower_csc_from_coo(n, rows, cols, vals)
    return Problem(n, cp, ri.astype(np.int32), vx, None)


def random_spd_pattern(n, density, seed, nrhs=1, dominance=1.0):
    """Random symmetric pattern with diagonally dominant values (SPD)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = rng.random((n, n)) < density
    low = np.tril(mask, -1)
    r, c = np.nonzero(low)
    w = rng.uniform(0.1, 1.0, size=r.size) * rng.choice([-1.0, 1.0], size=r.size)
    deg = np.zeros(n)
    np.add.at(deg, r, np.abs(w))
    np.add.at(deg, c, np.abs(w))
    rows = np.concatenate([r, np.arange(n)])
    cols = np.concatenate([c, np.arange(n)])
    vals = np.concatenate([w, deg + dominance])
    cp, ri, vx = lower_csc_from_coo(n, rows, cols, vals)
    perm = rng.permutation(n).astype(np.int32)
    rhs = np.asfortranarray(rng.standard_normal((n, nrhs))) if nrhs else None
    return Problem(n, cp, ri.astype(np.int32), vx, perm, rhs)


def dense_spd(n, seed, nrhs=1):
    """Dense SPD A = G G^T / n + I as a fully stored lower CSC."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((n, n))
    a = g @ g.T / max(n, 1) + np.eye(n)
    j, i = np.meshgrid(np.arange(n), np.arange(n))
    m = i >= j
    cp, ri, vx = lower_csc_from_coo(n, i[m], j[m], a[m])
    rhs = np.asfortranarray(rng.standard_normal((n, nrhs))) if nrhs else None
    return Problem(n, cp, ri.astype(np.int32), vx, None, rhs)
