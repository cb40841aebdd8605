"""GPU parity of the HIP factorization and solve with the CPU oracle, through
the C ABI, on seeded inputs that span several tiles, ragged tails, chains
split by the cap, amalgamated supernodes and the degenerate cases.

Bars: integer structure bit-exact (checked on the CPU); every entry of the
FP64 factor within |dL_ij| <= 1e-10 |L_ij| + 1e-13 sqrt(c_ii c_jj) / L_jj of
the oracle's (c = diagonal of P A P^T); explicit zeros of amalgamated storage
exactly zero; ||L L^T - P A P^T||_F / ||A||_F <= 1e-12; normwise backward
error of the solution <= 1e-14, and its distance to the oracle's solution
within cond(A) times the two backward errors (both are backward stable)."""
import numpy as np
import pytest

import oracle
from paper_1608_00044_amd import inputs, spchol
from tests.gpu_util import compare_factor, gpu_factor, say, torch_dev
from tests.helpers import load_fig1, spd_values_for_pattern

pytestmark = pytest.mark.gpu


def _case(name):
    if name.startswith("dense"):
        n = int(name[5:])
        return inputs.dense_spd(n, seed=n, nrhs=2), 150, 0.0
    if name.startswith("tridiag"):
        p = inputs.tridiag(int(name[7:]))
        p.rhs = np.asfortranarray(np.random.default_rng(1).standard_normal((p.n, 1)))
        return p, 150, 0.0
    if name == "fig1":
        fig = load_fig1()
        p = spd_values_for_pattern(fig["n"], fig["orig"], seed=2)
        p.rhs = np.asfortranarray(np.random.default_rng(2).standard_normal((p.n, 3)))
        return p, 150, 0.0
    if name.startswith("random"):
        seed = int(name[6:])
        rng = np.random.default_rng(seed)
        n = int(rng.integers(20, 400))
        return inputs.random_spd_pattern(n, float(rng.uniform(0.005, 0.05)), seed, nrhs=2), \
            int(rng.choice([4, 16, 150])), float(rng.choice([0.0, 0.2]))
    if name == "lap2d_64":
        return inputs.make_workload("lap2d_5pt_64"), 150, 0.0
    if name == "lap3d_12_amalg":
        return inputs.make_grid_problem("lap", (12, 12, 12), 5, sigma=1.0, shift=1e-6), 150, 0.1
    if name == "lap3d_20_cap32":
        return inputs.make_grid_problem("lap", (20, 20, 20), 6, sigma=1.0, shift=1e-6,
                                        nrhs=2), 32, 0.1
    if name == "lap3d_24":
        return inputs.make_grid_problem("lap", (24, 24, 24), 8, sigma=1.0, shift=1e-6), 150, 0.1
    if name == "lap2d_40_cap8":
        return inputs.make_grid_problem("lap", (40, 40), 9, sigma=0.5, shift=1e-3), 8, 0.3
    if name == "elast27_6":
        return inputs.make_grid_problem("27pt3", (6, 6, 6), 10, shift=1e-3, nrhs=2), 150, 0.1
    raise KeyError(name)


def _cond_bound(p):
    """Upper bound of the 2-norm condition number: ||A||_inf over a lower bound
    of lambda_min (the diagonal shift for the shifted Laplacians, whose graph
    Laplacian part is positive semidefinite; the exact value for small dense
    cases)."""
    shift = p.meta.get("shift") if p.meta else None
    a = inputs.dense_from_lower_csc(p.n, p.colptr, p.rowind, p.values) if p.n <= 2000 else None
    if a is not None:
        return float(np.linalg.cond(a))
    import scipy.sparse as sp

    A = sp.csc_matrix((p.values, p.rowind, p.colptr), shape=(p.n, p.n))
    A = A + sp.tril(A, -1).T
    return float(abs(A).sum(axis=1).max() / shift)


CASES = ["dense1", "dense2", "dense5", "dense63", "dense64", "dense65", "dense150", "dense151",
         "dense300", "tridiag1000", "fig1", "random1", "random2", "random3", "random4",
         "lap2d_64", "lap3d_12_amalg", "lap3d_20_cap32", "lap3d_24", "lap2d_40_cap8",
         "elast27_6"]


SUBSET = ("dense300", "fig1", "random3", "lap2d_64", "lap3d_20_cap32", "lap3d_24", "elast27_6")

# (case, schedule, order): every case in the default deterministic order
# (sched 0) and on the task queue (sched 2, atomic order); a subset in the
# atomic order level by level and with the lookahead (sched 1)
SCHED_CASES = ([(c, 0, 1) for c in CASES] + [(c, 0, 0) for c in SUBSET]
               + [(c, 1, 0) for c in SUBSET] + [(c, 2, 0) for c in CASES])


@pytest.mark.parametrize("name,sched,det", SCHED_CASES)
def test_factor_and_solve_parity(name, sched, det):
    torch = torch_dev()
    p, cap, ratio = _case(name)
    say("case", name, "sched", sched, "deterministic", det, "n", p.n, "nnz", p.nnz, "cap", cap,
        "ratio", ratio)
    sym, num, _ = gpu_factor(p, cap, ratio, sched, deterministic=det)
    assert num.status() == 0
    worst, rho, (osym, Lx, got) = compare_factor(p, num, cap, ratio, name)
    say("  worst/tol", worst, "residual", rho)
    assert worst <= 1.0
    assert rho <= 1e-12
    if p.rhs is not None:
        b = torch.from_numpy(np.ascontiguousarray(p.rhs)).to("cuda:0")
        x = num.solve(b if b.shape[1] > 1 else b[:, 0]).cpu().numpy().reshape(p.n, -1)
        xo = oracle.solve(p.n, osym, Lx, p.perm, p.rhs).reshape(p.n, -1)
        eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs, x)
        eta_o = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs, xo)
        say("  backward error", eta.max(), "oracle", eta_o.max())
        assert eta.max() <= 1e-14
        # both solutions are backward stable, so they agree to within
        # cond(A) * (eta + eta_oracle); cond(A) <= ||A||_inf / lambda_min
        kappa = _cond_bound(p)
        fwd = np.abs(x - xo).max() / np.abs(xo).max()
        say("  forward difference", fwd, "bound", 4 * kappa * (eta.max() + eta_o.max()))
        assert fwd <= max(1e-12, 4 * kappa * (eta.max() + eta_o.max()))
    num.free()
    sym.free()


def test_tridiag_closed_form_on_gpu():
    n = 777
    p = inputs.tridiag(n)
    sym, num, _ = gpu_factor(p)
    Sp, Si, Sx = num.export()
    i = np.arange(1, n + 1, dtype=np.float64)
    diag = Sx[Sp[:-1]]
    np.testing.assert_allclose(diag, np.sqrt((i + 1) / i), rtol=1e-14)
    # sub-diagonal: second stored entry of every column but the last
    sub = Sx[Sp[:-2] + 1]
    assert np.array_equal(Si[Sp[:-2] + 1], np.arange(1, n))
    np.testing.assert_allclose(sub, -np.sqrt(i[:-1] / (i[:-1] + 1)), rtol=1e-14)


@pytest.mark.parametrize("k", [1, 2, 30, 400])
def test_non_spd_reports_first_failing_column(k):
    torch = torch_dev()
    n = 400
    p = inputs.tridiag(n)
    vals = p.values.copy()
    vals[p.colptr[k - 1]] = (k - 1) / k - 0.5
    q = inputs.Problem(n, p.colptr, p.rowind, vals, None)
    sym, num, _ = gpu_factor(q)
    assert num.status() == k
    b = torch.ones(n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(spchol.SpcError) as e:
        num.solve(b)
    assert e.value.status == k


def test_non_spd_in_3d_parallel_schedule():
    """Two independent failures: the smallest failing permuted column is reported."""
    p = inputs.make_grid_problem("lap", (10, 10, 10), 3, sigma=1.0, shift=1e-3, nrhs=0)
    Cp, Ci, Cx, mp = oracle.permute(p.n, p.colptr, p.rowind, p.values, p.perm)
    vals = p.values.copy()
    # make two diagonal entries negative; find their permuted columns
    inv = np.argsort(mp)  # C position -> input entry
    cols = []
    for j in (137, 611):
        q = Cp[j]  # diagonal is the first entry of column j of C
        vals[inv[q]] = -1.0
        cols.append(j)
    q2 = inputs.Problem(p.n, p.colptr, p.rowind, vals, p.perm)
    Cp2, Ci2, Cx2, _ = oracle.permute(p.n, q2.colptr, q2.rowind, q2.values, q2.perm)
    osym = oracle.symbolic(p.n, Cp2, Ci2)
    ost, _ = oracle.factor(p.n, Cp2, Ci2, Cx2, osym)
    sym, num, _ = gpu_factor(q2, 150, 0.1)
    assert num.status() == ost == min(cols) + 1


@pytest.mark.parametrize("sched", [1, 2])
def test_non_spd_status_other_schedules(sched):
    """The failing column is reported the same way by every schedule."""
    n = 400
    p = inputs.tridiag(n)
    vals = p.values.copy()
    vals[p.colptr[29]] = 29 / 30 - 0.5
    sym, num, _ = gpu_factor(inputs.Problem(n, p.colptr, p.rowind, vals, None), sched=sched)
    assert num.status() == 30


def test_task_queue_refactor_resets_counters():
    """Two factorizations in a row through one task-queue plan: the dependency
    counters start over each time."""
    torch = torch_dev()
    p = inputs.make_grid_problem("lap", (14, 14, 14), 31, sigma=1.0, shift=1e-3, nrhs=0)
    sym, num, _ = gpu_factor(p, 150, 0.1, sched=2)
    assert num.status() == 0
    p2 = inputs.make_grid_problem("lap", (14, 14, 14), 32, sigma=1.0, shift=1e-3, nrhs=0)
    for _ in range(2):
        num.refactor(torch.from_numpy(p2.values).to("cuda:0"))
        assert num.status() == 0
        worst, rho, _ = compare_factor(p2, num, 150, 0.1, "refactor-sched2")
        assert worst <= 1.0 and rho <= 1e-12


def test_task_queue_bounded_wait_reports_timeout():
    """A dependency the host withholds (debug flag) never arrives: the bounded
    device wait ends the factorization with SPC_ERR_TIMEOUT, every worker
    exits, and the device stays usable."""
    torch = torch_dev()
    p = inputs.make_grid_problem("lap", (8, 8, 8), 5, sigma=1.0, shift=1e-3, nrhs=0)
    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sched=2, spin_limit=200000,
                         debug_flags=1)
    vals = torch.from_numpy(p.values).to("cuda:0")
    num = spchol.factor(sym, vals)
    assert num.status() == spchol.SPC_ERR_TIMEOUT
    with pytest.raises(spchol.SpcError) as e:
        num.solve(torch.ones(p.n, dtype=torch.float64, device="cuda:0"))
    assert e.value.status == spchol.SPC_ERR_TIMEOUT
    num.free()
    sym.free()
    sym2, num2, _ = gpu_factor(p, sched=2)
    assert num2.status() == 0


@pytest.mark.parametrize("nrhs", [1, 3])
def test_solve_bounded_wait_leaves_nan(nrhs):
    """The solves' level launches wait on device-side counts; with one count
    withheld (debug flag) every wait passes its bound (2 ms), every
    workgroup still exits, and the solution holds NaN instead of numbers
    computed from data that never arrived; the device stays usable."""
    torch = torch_dev()
    p = inputs.make_grid_problem("lap", (12, 12, 12), 5, sigma=1.0, shift=1e-3, nrhs=nrhs)
    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, spin_limit=2000, debug_flags=1)
    vals = torch.from_numpy(p.values).to("cuda:0")
    num = spchol.factor(sym, vals)
    assert num.status() == 0  # the level-set factorization has no waits
    b = torch.from_numpy(np.ascontiguousarray(p.rhs)).to("cuda:0")
    x = num.solve(b if nrhs > 1 else b[:, 0]).cpu().numpy()
    say("nrhs", nrhs, "NaN entries", int(np.isnan(x).sum()), "of", x.size)
    assert np.isnan(x).any()
    num.free()
    sym.free()
    sym2, num2, _ = gpu_factor(p)
    x2 = num2.solve(b if nrhs > 1 else b[:, 0]).cpu().numpy()
    eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs,
                                x2.reshape(p.n, -1))
    assert eta.max() <= 1e-14


def test_nan_value_reports_status():
    n = 50
    p = inputs.tridiag(n)
    vals = p.values.copy()
    vals[p.colptr[9]] = np.nan
    sym, num, _ = gpu_factor(inputs.Problem(n, p.colptr, p.rowind, vals, None))
    assert num.status() == 10


def test_refactor_and_multi_rhs():
    torch = torch_dev()
    p = inputs.make_grid_problem("lap", (16, 16, 16), 21, sigma=1.0, shift=1e-3, nrhs=4)
    sym, num, _ = gpu_factor(p, 150, 0.1)
    assert num.status() == 0
    p2 = inputs.make_grid_problem("lap", (16, 16, 16), 22, sigma=1.0, shift=1e-3, nrhs=4)
    assert np.array_equal(p2.colptr, p.colptr) and np.array_equal(p2.rowind, p.rowind)
    num.refactor(torch.from_numpy(p2.values).to("cuda:0"))
    assert num.status() == 0
    worst, rho, (osym, Lx, _) = compare_factor(p2, num, 150, 0.1, "refactor")
    assert worst <= 1.0 and rho <= 1e-12
    b = torch.from_numpy(np.ascontiguousarray(p2.rhs)).to("cuda:0")
    x = num.solve(b).cpu().numpy()
    xo = oracle.solve(p2.n, osym, Lx, p2.perm, p2.rhs)
    tol = 4 * _cond_bound(p2) * 1e-15
    np.testing.assert_allclose(x, xo, rtol=0, atol=tol * np.abs(xo).max())
    assert oracle.backward_error(p2.n, p2.colptr, p2.rowind, p2.values, p2.rhs, x).max() <= 1e-14
    # in-place solve (x aliases b): the solve's sums have one fixed order, so
    # the same bits
    bb = b.t().contiguous().t()
    num.solve(bb, x=bb)
    assert np.array_equal(bb.cpu().numpy(), x)


def test_empty_matrix():
    torch = torch_dev()
    sym = spchol.analyze(0, [0], [])
    num = spchol.factor(sym, torch.zeros(1, dtype=torch.float64, device="cuda:0"))
    assert num.status() == 0
    num.free()
    sym.free()


def test_symbolic_free_refuses_while_factor_alive():
    p = inputs.tridiag(10)
    sym, num, _ = gpu_factor(p)
    with pytest.raises(spchol.SpcError) as e:
        sym.free()
    assert e.value.status == spchol.SPC_ERR_BUSY
    num.free()
    sym.free()


def test_memory_budget_rejects_large_factor():
    torch = torch_dev()
    p = inputs.make_grid_problem("lap", (16, 16, 16), 1, sigma=1.0, shift=1e-3, nrhs=0)
    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, mem_budget_bytes=1 << 20)
    with pytest.raises(spchol.SpcError) as e:
        spchol.factor(sym, torch.from_numpy(p.values).to("cuda:0"))
    assert e.value.status == spchol.SPC_ERR_OOM


def test_solve_graph_replays_match():
    """The solve sweeps replay from a captured graph: repeated solves, with
    other right-hand sides and a refactorization between them, all give the
    oracle's answer, and (deterministic order) the same bits every time."""
    torch = torch_dev()
    p = inputs.make_grid_problem("lap", (14, 14, 14), 31, sigma=1.0, shift=1e-3, nrhs=3)
    sym, num, vals = gpu_factor(p, 150, 0.1)
    out = oracle.run(p, cap=150, ratio=0.1)
    xo = out["x"]
    b = torch.from_numpy(np.ascontiguousarray(p.rhs)).to("cuda:0")
    scale = np.abs(xo).max()
    other = torch.randn(p.n, dtype=torch.float64, device="cuda:0")
    first = None
    for rep in range(5):
        x = num.solve(b).cpu().numpy()
        np.testing.assert_allclose(x, xo, rtol=0, atol=1e-9 * scale)
        num.solve(other)                       # a different graph (nrhs = 1)
        x1 = num.solve(b[:, 1]).cpu().numpy()  # and a one-column replay
        np.testing.assert_allclose(x1, xo[:, 1], rtol=0, atol=1e-9 * scale)
        if first is None:
            first = (x, x1)
        assert np.array_equal(x, first[0]) and np.array_equal(x1, first[1])
        if rep == 2:
            num.refactor(vals)                 # same values: same factor
            assert num.status() == 0
    num.free()
    sym.free()


@pytest.mark.parametrize("k", [1, 7, 8, 9, 20])
def test_solve_right_hand_side_groups(k):
    """Right-hand sides go through the solve kernels in groups of eight: every
    column of a ragged last group matches the one-column solve of the same
    right-hand side, and all are backward stable."""
    torch = torch_dev()
    p = inputs.make_grid_problem("lap", (14, 14, 14), 51, sigma=1.0, shift=1e-3, nrhs=0)
    sym, num, _ = gpu_factor(p, 150, 0.1)
    assert num.status() == 0
    B = np.asfortranarray(np.random.default_rng(k).standard_normal((p.n, k)))
    x = num.solve(torch.from_numpy(B).to("cuda:0")).cpu().numpy().reshape(p.n, k)
    eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, B, x)
    assert eta.max() <= 1e-14
    for c in (0, k - 1):
        xc = num.solve(torch.from_numpy(np.ascontiguousarray(B[:, c])).to("cuda:0")).cpu().numpy()
        np.testing.assert_allclose(x[:, c], xc, rtol=0, atol=1e-12 * np.abs(xc).max())


@pytest.mark.parametrize("sched,det", [(0, 1), (0, 0), (1, 0)])
def test_factor_graph_replays_match_direct_launches(sched, det):
    """The level-set factorization (sched 1: with the lookahead's second
    stream joined into the capture) is captured into a graph on the first
    factorization and replayed after; every replay (with eager work between)
    and a directly launched factorization (per-launch timing on) agree, bit
    for bit in the deterministic order and to rounding in the atomic one, and
    the last replay meets the parity bars."""
    torch = torch_dev()
    p = inputs.make_grid_problem("lap", (16, 16, 16), 71, sigma=1.0, shift=1e-3, nrhs=0)
    sym, num, vals = gpu_factor(p, 150, 0.1, sched, deterministic=det)
    L1 = num.export()[2]
    scale = np.abs(L1).max()

    def same(L):
        if det:
            assert np.array_equal(L, L1)
        else:
            np.testing.assert_allclose(L, L1, rtol=0, atol=1e-13 * scale)

    for _ in range(3):
        torch.ones(1000, device="cuda:0").sum().item()  # eager work between replays
        num.refactor(vals)
        same(num.export()[2])
    num.set_timing(True)
    num.refactor(vals)
    same(num.export()[2])
    assert num.timing()["update"]["launches"] > 0
    num.set_timing(False)
    num.refactor(vals)
    worst, rho, _ = compare_factor(p, num, 150, 0.1, "graph replay")
    assert worst <= 1.0 and rho <= 1e-12


@pytest.mark.parametrize("chunk,precision", [(8, 0), (32, 0), (8, 1), (32, 1)])
def test_update_chunk_shapes_give_the_same_bits(chunk, precision):
    """The update tiles' K chunk (a tile shape the batch autotuner searches)
    changes only how the source panel is staged: the products and their
    order are the same, so the factor has the same bits."""
    p = inputs.make_grid_problem("lap", (20, 20, 20), 6, sigma=1.0, shift=1e-6, nrhs=0)
    say("chunk", chunk, "precision", precision, "n", p.n)
    sym, num, _ = gpu_factor(p, 150, 0.1, precision=precision)
    symc, numc, _ = gpu_factor(p, 150, 0.1, precision=precision, upd_chunk=chunk)
    assert num.status() == 0 and numc.status() == 0
    assert np.array_equal(numc.export()[2], num.export()[2])
    for o in (num, numc, sym, symc):
        o.free()
