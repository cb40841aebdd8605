"""Shared test helpers: fixture loaders and small brute-force references.

Nothing here imports the HIP library; the brute-force routines are
independent of both the oracle and the library (they are the pins)."""
from __future__ import annotations

import os

import numpy as np

from paper_1608_00044_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_fig1():
    """Parse tests/golden/fig1_structure.txt -> dict with n, supernodes,
    original (set of (row, col)), fill (set), etree {child: parent} (1-based)."""
    sn, orig, fill, etree = [], set(), set(), {}
    with open(os.path.join(GOLDEN, "fig1_structure.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            tag, vals = line[0], [int(v) for v in line[1:]]
            if tag == "supernode":
                sn.append((vals[0], vals[1], vals[2]))
            elif tag in ("block", "fill"):
                c0, c1, r0, r1 = vals
                tgt = orig if tag == "block" else fill
                for c in range(c0, c1 + 1):
                    for r in range(r0, r1 + 1):
                        tgt.add((r, c))
            elif tag == "etree":
                etree[vals[0]] = vals[1]
    # diagonal blocks are dense lower triangles of original entries
    for _, a, b in sn:
        for c in range(a, b + 1):
            for r in range(c, b + 1):
                orig.add((r, c))
    n = max(b for _, _, b in sn) + 1
    return dict(n=n, supernodes=sn, orig=orig, fill=fill, etree=etree)


def spd_values_for_pattern(n, entries, seed=0):
    """Diagonally dominant SPD values on a given lower pattern -> inputs.Problem
    in natural order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    entries = sorted(set(entries) | {(i, i) for i in range(n)})
    rows = np.array([e[0] for e in entries])
    cols = np.array([e[1] for e in entries])
    off = rows != cols
    vals = np.zeros(len(entries))
    vals[off] = -rng.uniform(0.1, 1.0, size=off.sum())
    deg = np.zeros(n)
    np.add.at(deg, rows[off], -vals[off])
    np.add.at(deg, cols[off], -vals[off])
    vals[~off] = deg[rows[~off]] + 1.0
    cp, ri, vx = inputs.lower_csc_from_coo(n, rows, cols, vals)
    return inputs.Problem(n, cp, ri.astype(np.int32), vx, None)


def elimination_game(n, pattern):
    """Boolean Gaussian elimination on a symmetric pattern (set of (i, j), i >= j,
    in the already-permuted order).  Returns (struct, parent, colcount) where
    struct[j] is the sorted row list of column j of L."""
    adj = [set() for _ in range(n)]
    for i, j in pattern:
        if i != j:
            adj[i].add(j)
            adj[j].add(i)
    struct = []
    for j in range(n):
        later = sorted(v for v in adj[j] if v > j)
        struct.append([j] + later)
        for a in later:  # eliminating j makes its later neighbours a clique
            for b in later:
                if a != b:
                    adj[a].add(b)
    parent = [s[1] if len(s) > 1 else -1 for s in struct]
    cc = [len(s) for s in struct]
    return struct, parent, cc


def alg1_dense(a):
    """Algorithm 1 of the paper (Section II-A), column by column, in plain loops:
    l_jj = sqrt(a_jj); l_ij = a_ij / l_jj; then a_ik -= l_ij l_kj for k > j, i >= k."""
    a = np.array(a, dtype=np.float64)
    n = a.shape[0]
    L = np.zeros_like(a)
    for j in range(n):
        L[j, j] = np.sqrt(a[j, j])
        for i in range(j + 1, n):
            L[i, j] = a[i, j] / L[j, j]
        for k in range(j + 1, n):
            for i in range(k, n):
                a[i, k] = a[i, k] - L[i, j] * L[k, j]
    return L


def csc_to_dense_lower(n, Lp, Li, Lx):
    L = np.zeros((n, n))
    for j in range(n):
        for p in range(Lp[j], Lp[j + 1]):
            L[Li[p], j] = Lx[p]
    return L


def refusal_case(y):
    """Pattern for the refused-then-accepted amalgamation case (22 columns):
    columns 2..21 a dense block (supernode pp, 20 columns, nothing below);
    column 1 (supernode p) with rows {1} + S1, |S1| = 11, min S1 = 2, so
    colcount 12 and parent 2; column 0 (supernode c) with rows {0, 1} plus
    y - 2 rows of S1, so colcount y and parent 1."""
    n = 22
    S1 = [2, 3, 5, 7, 8, 10, 12, 14, 16, 18, 21]
    S0 = [1] + S1[: y - 2]
    ent = [(i, i) for i in range(n)] + [(r, 0) for r in S0] + [(r, 1) for r in S1]
    ent += [(i, j) for j in range(2, n) for i in range(j + 1, n)]
    return spd_values_for_pattern(n, ent, seed=y)
