"""Pins for the CPU oracle: each check ties it to something other than itself --
a worked example printed in the paper, closed forms, brute force on tiny
inputs, LAPACK, or invariants the mathematics fixes."""
import numpy as np
import pytest

import oracle
from paper_1608_00044_amd import inputs
from tests.helpers import (alg1_dense, csc_to_dense_lower, elimination_game, load_fig1,
                           refusal_case, spd_values_for_pattern)


# ---------------------------------------------------------------------------
# Fig. 1 worked example (Section II-B)
# ---------------------------------------------------------------------------

def _fig1_oracle():
    fig = load_fig1()
    p = spd_values_for_pattern(fig["n"], fig["orig"], seed=11)
    Cp, Ci, Cx, _ = oracle.permute(p.n, p.colptr, p.rowind, p.values, None)
    sym = oracle.symbolic(p.n, Cp, Ci)
    return fig, p, (Cp, Ci, Cx), sym


def test_fig1_structure_of_L():
    fig, p, _, sym = _fig1_oracle()
    got = {(int(sym.Li[q]), j) for j in range(p.n) for q in range(sym.Lp[j], sym.Lp[j + 1])}
    want = fig["orig"] | fig["fill"]
    assert got == want
    assert sym.nnz == 155
    # fill-in appears only where the figure marks it: in supernode 8, rows 25, 26, 28
    assert got - fig["orig"] == fig["fill"]


def test_fig1_supernodes_and_supernodal_etree():
    fig, p, _, sym = _fig1_oracle()
    sn = oracle.supernodes(p.n, sym.parent, sym.colcount, cap=150)
    want = [a for _, a, _ in fig["supernodes"]] + [p.n]
    assert sn.tolist() == want  # the paper finds ten supernodes
    sp = oracle.supernodal_parent(sym.parent, sn)
    got = {s + 1: int(sp[s]) + 1 for s in range(len(sp)) if sp[s] >= 0}
    assert got == fig["etree"]
    assert sp[-1] == -1


def test_fig1_etree_definition():
    """parent(j) is the first off-diagonal nonzero row of column j of L."""
    fig, p, _, sym = _fig1_oracle()
    L = fig["orig"] | fig["fill"]
    for j in range(p.n):
        below = sorted(r for r, c in L if c == j and r > j)
        assert sym.parent[j] == (below[0] if below else -1)
        assert sym.colcount[j] == len(below) + 1


# ---------------------------------------------------------------------------
# brute-force elimination game
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_symbolic_vs_elimination_game(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 13))
    p = inputs.random_spd_pattern(n, density=float(rng.uniform(0.05, 0.5)), seed=seed)
    Cp, Ci, Cx, _ = oracle.permute(n, p.colptr, p.rowind, p.values, p.perm)
    pattern = {(int(Ci[q]), j) for j in range(n) for q in range(Cp[j], Cp[j + 1])}
    struct, parent, cc = elimination_game(n, pattern)
    sym = oracle.symbolic(n, Cp, Ci)
    assert sym.parent.tolist() == parent
    assert sym.colcount.tolist() == cc
    for j in range(n):
        assert sym.Li[sym.Lp[j]:sym.Lp[j + 1]].tolist() == struct[j]


# ---------------------------------------------------------------------------
# closed forms of the symbolic structure
# ---------------------------------------------------------------------------

def _sym_of(p):
    Cp, Ci, Cx, _ = oracle.permute(p.n, p.colptr, p.rowind, p.values, p.perm)
    return oracle.symbolic(p.n, Cp, Ci), (Cp, Ci, Cx)


@pytest.mark.parametrize("n", [1, 2, 3, 10, 301])
def test_tridiagonal_closed_form(n):
    sym, _ = _sym_of(inputs.tridiag(n))
    assert sym.parent.tolist() == list(range(1, n)) + [-1]
    assert sym.colcount.tolist() == [2] * (n - 1) + [1]
    sn = oracle.supernodes(n, sym.parent, sym.colcount, cap=150)
    # {0}, ..., {n-3}, {n-2, n-1}
    want = list(range(0, n - 1)) + [n] if n >= 2 else [0, 1]
    assert sn.tolist() == want


def test_diagonal_closed_form():
    n = 17
    cp, ri, vx = inputs.lower_csc_from_coo(n, np.arange(n), np.arange(n), np.full(n, 3.0))
    p = inputs.Problem(n, cp, ri.astype(np.int32), vx, None)
    sym, C = _sym_of(p)
    assert (sym.parent == -1).all() and (sym.colcount == 1).all()
    st, Lx = oracle.factor(n, *C, sym)
    assert st == 0 and np.allclose(Lx, np.sqrt(3.0), rtol=0, atol=0)


def test_arrow_closed_form():
    n = 12
    rows = np.concatenate([np.arange(n), np.full(n - 1, n - 1)])
    cols = np.concatenate([np.arange(n), np.arange(n - 1)])
    vals = np.concatenate([np.full(n, float(n)), -np.ones(n - 1)])
    cp, ri, vx = inputs.lower_csc_from_coo(n, rows, cols, vals)
    sym, _ = _sym_of(inputs.Problem(n, cp, ri.astype(np.int32), vx, None))
    assert sym.parent.tolist() == [n - 1] * (n - 1) + [-1]
    assert sym.colcount.tolist() == [2] * (n - 1) + [1]
    sn = oracle.supernodes(n, sym.parent, sym.colcount, cap=150)
    assert sn.tolist() == list(range(n - 1)) + [n]


@pytest.mark.parametrize("n,cap,widths", [(40, 150, [40]), (300, 150, [150, 150]),
                                          (301, 150, [101, 100, 100]), (7, 3, [3, 2, 2])])
def test_dense_one_chain_split_by_cap(n, cap, widths):
    p = inputs.dense_spd(n, seed=n)
    sym, _ = _sym_of(p)
    assert sym.parent.tolist() == list(range(1, n)) + [-1]
    assert sym.colcount.tolist() == list(range(n, 0, -1))
    sn = oracle.supernodes(n, sym.parent, sym.colcount, cap=cap)
    assert np.diff(sn).tolist() == widths


@pytest.mark.parametrize("dims", [(9, 9), (16, 16), (6, 6, 6), (8, 8, 8)])
def test_top_separator_is_dense(dims):
    """Under nested dissection the last plane (s = k^(d-1) nodes for a k^d grid)
    is the top separator; its columns of L are dense: colcount(j) = n - j."""
    p = inputs.make_grid_problem("lap", dims, seed=1, shift=1e-3, nrhs=0)
    sym, _ = _sym_of(p)
    n = p.n
    s = int(np.prod(dims)) // max(dims)
    tail = sym.colcount[n - s:]
    assert tail.tolist() == list(range(s, 0, -1))


# ---------------------------------------------------------------------------
# permutation
# ---------------------------------------------------------------------------

def test_permute_matches_dense():
    p = inputs.random_spd_pattern(23, 0.2, seed=5)
    Cp, Ci, Cx, mp = oracle.permute(p.n, p.colptr, p.rowind, p.values, p.perm)
    want = inputs.dense_from_lower_csc(p.n, p.colptr, p.rowind, p.values, perm=p.perm)
    got = inputs.dense_from_lower_csc(p.n, Cp, Ci, Cx)
    assert np.array_equal(got, want)
    for j in range(p.n):
        col = Ci[Cp[j]:Cp[j + 1]]
        assert (np.diff(col) > 0).all() and (col >= j).all()
    assert np.array_equal(Cx[mp], p.values)


def test_validate_rejects_bad_patterns():
    n = 4
    cp = np.array([0, 2, 3, 4, 5])
    assert oracle.validate(n, cp, np.array([0, 1, 1, 2, 3])) == 0
    assert oracle.validate(n, cp, np.array([1, 0, 1, 2, 3])) == -2  # unsorted
    assert oracle.validate(n, cp, np.array([0, 0, 1, 2, 3])) == -2  # duplicate
    assert oracle.validate(n, cp, np.array([0, 1, 0, 2, 3])) == -2  # upper entry
    assert oracle.validate(n, cp, np.array([0, 1, 1, 2, 4])) == -2  # out of range
    assert oracle.validate(n, cp, np.array([0, 1, 1, 2, 3]), perm=np.array([0, 1, 1, 2])) == -1


# ---------------------------------------------------------------------------
# numeric factor
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 5, 17, 40])
def test_dense_factor_vs_alg1_and_lapack(n):
    p = inputs.dense_spd(n, seed=100 + n)
    sym, C = _sym_of(p)
    st, Lx = oracle.factor(n, *C, sym)
    assert st == 0
    L = csc_to_dense_lower(n, sym.Lp, sym.Li, Lx)
    A = inputs.dense_from_lower_csc(n, p.colptr, p.rowind, p.values)
    np.testing.assert_allclose(L, alg1_dense(A), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(L, np.linalg.cholesky(A), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 50, 1000])
def test_tridiag_closed_form_factor(n):
    """tridiag(-1, 2, -1): L_ii = sqrt((i+1)/i), L_{i+1,i} = -sqrt(i/(i+1)), 1-based."""
    sym, C = _sym_of(inputs.tridiag(n))
    st, Lx = oracle.factor(n, *C, sym)
    assert st == 0
    i = np.arange(1, n + 1, dtype=np.float64)
    diag = Lx[sym.Lp[:-1]]
    np.testing.assert_allclose(diag, np.sqrt((i + 1) / i), rtol=1e-14)
    sub = Lx[sym.Lp[:-2] + 1]
    np.testing.assert_allclose(sub, -np.sqrt(i[:-1] / (i[:-1] + 1)), rtol=1e-14)


def test_manufactured_factor_on_fig1_pattern():
    """Choose L0 on the Fig. 1 structure, set A = L0 L0^T; the factor must return L0."""
    fig = load_fig1()
    n = fig["n"]
    rng = np.random.default_rng(3)
    L0 = np.zeros((n, n))
    for r, c in fig["orig"] | fig["fill"]:
        L0[r, c] = rng.uniform(1.0, 2.0) if r == c else rng.uniform(-0.5, 0.5)
    A = L0 @ L0.T
    cp, ri, vx = inputs.lower_csc_from_dense(A)
    p = inputs.Problem(n, cp, ri.astype(np.int32), vx, None)
    sym, C = _sym_of(p)
    st, Lx = oracle.factor(n, *C, sym)
    assert st == 0
    L = csc_to_dense_lower(n, sym.Lp, sym.Li, Lx)
    np.testing.assert_allclose(L, L0, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("k", [1, 2, 7, 30])
def test_non_spd_status(k):
    """tridiag(-1,2,-1) with a_kk = (k-1)/k - delta makes the k-th pivot -delta."""
    n = 40
    p = inputs.tridiag(n)
    vals = p.values.copy()
    vals[p.colptr[k - 1]] = (k - 1) / k - 0.5
    sym, C = _sym_of(inputs.Problem(n, p.colptr, p.rowind, vals, None))
    st, _ = oracle.factor(n, *C, sym)
    assert st == k


def test_nan_input_status():
    n = 10
    p = inputs.tridiag(n)
    vals = p.values.copy()
    vals[p.colptr[4]] = np.nan
    sym, C = _sym_of(inputs.Problem(n, p.colptr, p.rowind, vals, None))
    st, _ = oracle.factor(n, *C, sym)
    assert st == 5


def test_residual_matches_dense_and_invariant():
    p = inputs.make_grid_problem("lap", (12, 12), seed=3, sigma=1.0, shift=1e-3)
    sym, C = _sym_of(p)
    st, Lx = oracle.factor(p.n, *C, sym)
    assert st == 0
    rho = oracle.residual_exact(p.n, *C, sym, Lx)
    assert rho <= 1e-12
    # on a factor perturbed well above rounding, the residual equals the dense one
    Lp_ = Lx * (1 + 1e-7 * np.random.default_rng(1).standard_normal(Lx.size))
    L = csc_to_dense_lower(p.n, sym.Lp, sym.Li, Lp_)
    Cd = inputs.dense_from_lower_csc(p.n, *C)
    want = np.linalg.norm(L @ L.T - Cd) / np.linalg.norm(Cd)
    np.testing.assert_allclose(oracle.residual_exact(p.n, *C, sym, Lp_), want, rtol=1e-6)
    # a planted mistake (one entry off by 1e-6) must be seen by the residual
    Lbad = Lx.copy()
    Lbad[len(Lbad) // 2] += 1e-6
    assert oracle.residual_exact(p.n, *C, sym, Lbad) > 1e-9
    z = np.random.default_rng(0).standard_normal((p.n, 8))
    est = oracle.residual_probe(p.n, *C, sym, Lx, z)
    assert est <= 1e-12


def test_cfg1_oracle_residual():
    p = inputs.make_workload("lap2d_5pt_64")
    out = oracle.run(p)
    assert out["status"] == 0
    rho = oracle.residual_exact(p.n, *out["C"], out["sym"], out["Lx"])
    assert rho <= 1e-12
    eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs, out["x"])
    assert eta.max() <= 1e-14


# ---------------------------------------------------------------------------
# solve
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 3, 64, 500])
def test_solve_tridiag_closed_form_inverse(n):
    """(A^{-1})_ij = min(i,j) (n+1-max(i,j)) / (n+1) for tridiag(-1,2,-1), 1-based."""
    p = inputs.tridiag(n)
    sym, C = _sym_of(p)
    st, Lx = oracle.factor(n, *C, sym)
    i = np.arange(1, n + 1)
    Ainv = np.minimum.outer(i, i) * (n + 1 - np.maximum.outer(i, i)) / (n + 1)
    b = np.random.default_rng(n).standard_normal((n, 3))
    x = oracle.solve(n, sym, Lx, None, b)
    np.testing.assert_allclose(x, Ainv @ b, rtol=1e-10, atol=1e-12 * np.abs(Ainv @ b).max())


def test_solve_manufactured_permuted():
    p = inputs.random_spd_pattern(60, 0.1, seed=9)
    x_true = np.random.default_rng(1).standard_normal((p.n, 2))
    b = inputs.dense_from_lower_csc(p.n, p.colptr, p.rowind, p.values) @ x_true
    out = oracle.run(inputs.Problem(p.n, p.colptr, p.rowind, p.values, p.perm, b))
    np.testing.assert_allclose(out["x"], x_true, rtol=1e-11, atol=1e-12)
    eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, b, out["x"])
    assert eta.max() <= 1e-15


def test_symv_and_backward_error_vs_numpy():
    p = inputs.random_spd_pattern(30, 0.3, seed=2)
    A = inputs.dense_from_lower_csc(p.n, p.colptr, p.rowind, p.values)
    z = np.random.default_rng(4).standard_normal((p.n, 2))
    np.testing.assert_allclose(oracle.symv(p.n, p.colptr, p.rowind, p.values, z), A @ z,
                               rtol=1e-14, atol=1e-14)
    x = z + 1e-3
    eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, z, x)
    r = z - A @ x
    want = np.abs(r).max(0) / (np.abs(A).sum(1).max() * np.abs(x).max(0) + np.abs(z).max(0))
    np.testing.assert_allclose(eta, want, rtol=1e-13)


# ---------------------------------------------------------------------------
# amalgamation (rule is a reading; pinned by invariants and hand-worked cases)
# ---------------------------------------------------------------------------

def _stored_counts(sn, sym):
    """Per column: stored count (last - j + 1) + r_last for the given partition."""
    out = np.zeros(sym.n, dtype=np.int64)
    for s in range(len(sn) - 1):
        a, b = sn[s], sn[s + 1] - 1
        r = sym.colcount[b] - 1
        for j in range(a, b + 1):
            out[j] = (b - j + 1) + r
    return out


@pytest.mark.parametrize("dims,ratio,cap", [((16, 16), 0.1, 150), ((8, 8, 8), 0.1, 150),
                                            ((10, 10, 10), 0.3, 64), ((20, 20), 0.05, 8)])
def test_amalgamation_invariants(dims, ratio, cap):
    p = inputs.make_grid_problem("lap", dims, seed=4, sigma=1.0, shift=1e-6, nrhs=0)
    sym, _ = _sym_of(p)
    sn0 = oracle.supernodes(p.n, sym.parent, sym.colcount, cap)
    sn = oracle.amalgamate(p.n, sym.parent, sym.colcount, sn0, cap, ratio)
    assert sn[0] == 0 and sn[-1] == p.n and (np.diff(sn) > 0).all()
    assert np.diff(sn).max() <= cap
    assert set(sn.tolist()) <= set(sn0.tolist())  # only whole supernodes merge
    assert len(sn) <= len(sn0)
    stored = _stored_counts(sn, sym)
    exact = sym.colcount.astype(np.int64)
    assert (stored >= exact).all()  # stored structure contains the exact one
    # each merged supernode obeys z / T <= ratio
    for s in range(len(sn) - 1):
        a, b = sn[s], sn[s + 1]
        if set(range(a + 1, b)) & set(sn0.tolist()):
            z = int((stored[a:b] - exact[a:b]).sum())
            T = int(stored[a:b].sum())
            assert z <= ratio * T
    # stored structure of each column contains its exact row set
    owner = np.repeat(np.arange(len(sn) - 1), np.diff(sn))
    for j in range(p.n):
        s = owner[j]
        last = sn[s + 1] - 1
        rows = set(range(j, last + 1)) | set(sym.Li[sym.Lp[last] + 1:sym.Lp[last + 1]].tolist())
        assert set(sym.Li[sym.Lp[j]:sym.Lp[j + 1]].tolist()) <= rows


def test_amalgamation_hand_worked():
    """Hand-worked: the arrow matrix's last two columns form {n-2, n-1}; the
    singleton {n-3} has exact count 2 and, merged, would store 3 + 0: z = 1,
    T = 3 + 2 + 1 = 6 -> z/T = 1/6.  At ratio 0.2 it merges, at 0.1 it does not.
    Repeating, {n-4} would give z = 1 + 2, T = 10 -> 0.3 (refused at 0.2)."""
    n = 8
    rows = np.concatenate([np.arange(n), np.full(n - 1, n - 1)])
    cols = np.concatenate([np.arange(n), np.arange(n - 1)])
    vals = np.concatenate([np.full(n, float(n)), -np.ones(n - 1)])
    cp, ri, vx = inputs.lower_csc_from_coo(n, rows, cols, vals)
    sym, _ = _sym_of(inputs.Problem(n, cp, ri.astype(np.int32), vx, None))
    sn0 = oracle.supernodes(n, sym.parent, sym.colcount, 150)
    assert sn0.tolist() == [0, 1, 2, 3, 4, 5, 6, 8]
    assert oracle.amalgamate(n, sym.parent, sym.colcount, sn0, 150, 0.1).tolist() == sn0.tolist()
    assert oracle.amalgamate(n, sym.parent, sym.colcount, sn0, 150, 0.2).tolist() == \
        [0, 1, 2, 3, 4, 5, 8]
    # cap 2 forbids the merge whatever the ratio
    assert oracle.amalgamate(n, sym.parent, sym.colcount, sn0, 2, 0.9).tolist() == sn0.tolist()


@pytest.mark.parametrize("y,expect", [(8, [0, 22]), (5, [0, 1, 22]), (11, [0, 22])])
def test_amalgamation_refused_then_accepted(y, expect):
    """Hand-worked at ratio 0.1 (a merged column j stores
    last(parent) - j + 1 + r_parent rows; z and T summed over the merged
    supernode, the parent's own z carried along):
    pass 1, c into p: stored(0) = 2 + 11 = 13 against colcount y, so
    z = 13 - y, T = 13 + 12 = 25, bar 2.5: for y <= 10 c is refused.
    Later in pass 1, p into pp: stored(1) = 21, z = 21 - 12 = 9,
    T = 210 + 21 = 231, bar 23.1: merged.
    Pass 2, c into the grown parent: stored(0) = 22, z = 9 + (22 - y),
    T = 231 + 22 = 253, bar 25.3: y = 8 gives 23 (merged: one supernode of
    22 columns); y = 5 gives 26 (refused, although c's own zeros, 17, are
    under the bar: the parent's zeros count too).  Without repeated passes
    y = 8 would stay apart.
    y = 11: pass 1 merges c into p (z = 2, T = 25), then {0, 1} into pp with
    both columns recounted against pp: z = (22 - 11) + (21 - 12) = 20,
    T = 210 + 22 + 21 = 253: one supernode."""
    p = refusal_case(y)
    sym, _ = _sym_of(p)
    assert sym.parent[0] == 1 and sym.parent[1] == 2
    assert sym.colcount[0] == y and sym.colcount[1] == 12 and sym.colcount[2] == 20
    sn0 = oracle.supernodes(p.n, sym.parent, sym.colcount, 150)
    assert sn0.tolist() == [0, 1, 2, 22]
    assert oracle.amalgamate(p.n, sym.parent, sym.colcount, sn0, 150, 0.1).tolist() == expect


def test_residual_probe_against_dense_and_exact():
    """The 8-probe estimate ||(L L^T - C) Z||_F / ||C Z||_F, written out densely
    with numpy for the same probes, equals the oracle's; its square has
    expectation rho^2 (E ||E z||^2 = ||E||_F^2 for Gaussian z), so eight probes
    land within a factor of 3 of the exact rho; a planted error in L raises it."""
    p = inputs.make_grid_problem("lap", (12, 12), seed=3, sigma=1.0, shift=1e-3)
    sym, C = _sym_of(p)
    st, Lx = oracle.factor(p.n, *C, sym)
    assert st == 0
    Lp_ = Lx * (1 + 1e-7 * np.random.default_rng(1).standard_normal(Lx.size))
    z = np.random.default_rng(0).standard_normal((p.n, 8))
    L = csc_to_dense_lower(p.n, sym.Lp, sym.Li, Lp_)
    Cd = inputs.dense_from_lower_csc(p.n, *C)
    dense = np.linalg.norm((L @ L.T - Cd) @ z) / np.linalg.norm(Cd @ z)
    est = oracle.residual_probe(p.n, *C, sym, Lp_, z)
    np.testing.assert_allclose(est, dense, rtol=1e-6)
    rho = oracle.residual_exact(p.n, *C, sym, Lp_)
    assert rho / 3 <= est <= 3 * rho
    Lbad = Lx.copy()
    Lbad[len(Lbad) // 2] += 1e-6
    assert oracle.residual_probe(p.n, *C, sym, Lbad, z) > 1e-9
    assert oracle.residual_probe(p.n, *C, sym, Lx, z) <= 1e-12
