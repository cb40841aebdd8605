"""GPU checks of the deterministic contribution order (the default): every
target supernode receives its update contributions in one fixed order
(level by level, and inside a level the sources in increasing order, the
non-decreasing (target, source) order of Section III-D), and the solves'
sums have fixed orders, so a factorization and a solve give the same bits
on every run; the atomic order (deterministic = 0) agrees with it to
rounding.  Also the task queue's execution log (Section IV): with one, two
or all workers every task starts after each task it depends on has
finished, and the factor meets the parity bars."""
import numpy as np
import pytest

from paper_1608_00044_amd import inputs, spchol
from tests.gpu_util import compare_factor, gpu_factor, say, torch_dev

pytestmark = pytest.mark.gpu


def _problem(name):
    if name == "lap3d_24":
        return inputs.make_grid_problem("lap", (24, 24, 24), 8, sigma=1.0, shift=1e-6,
                                        nrhs=3), 150, 0.1
    if name == "lap2d_64":
        return inputs.make_workload("lap2d_5pt_64"), 150, 0.0
    if name == "elast27_7":
        return inputs.make_grid_problem("27pt3", (7, 7, 7), 10, shift=1e-3, nrhs=2), 150, 0.1
    if name == "lap3d_20_cap32":
        return inputs.make_grid_problem("lap", (20, 20, 20), 6, sigma=1.0, shift=1e-6,
                                        nrhs=2), 32, 0.1
    raise KeyError(name)


@pytest.mark.parametrize("name", ["lap3d_24", "lap2d_64", "elast27_7", "lap3d_20_cap32"])
@pytest.mark.parametrize("precision", [0, 1])
def test_factor_and_solve_are_bit_identical(name, precision):
    torch = torch_dev()
    p, cap, ratio = _problem(name)
    say("case", name, "precision", precision, "n", p.n)
    sym, num, vals = gpu_factor(p, cap, ratio, precision=precision)
    assert num.status() == 0
    L0 = num.export()[2]
    b = torch.from_numpy(np.ascontiguousarray(p.rhs)).to("cuda:0")
    x0 = num.solve(b).cpu().numpy()
    # a second numeric object, refactorizations with eager work between them
    sym2, num2, _ = gpu_factor(p, cap, ratio, precision=precision)
    for rep in range(3):
        torch.randn(4096, device="cuda:0").sum().item()
        num2.refactor(vals)
        assert num2.status() == 0
        assert np.array_equal(num2.export()[2], L0), "factor differs on repeat %d" % rep
        assert np.array_equal(num2.solve(b).cpu().numpy(), x0), "solve differs on repeat %d" % rep
    if precision == 0:
        worst, rho, _ = compare_factor(p, num, cap, ratio, name)
        say("  worst/tol", worst, "residual", rho)
        assert worst <= 1.0 and rho <= 1e-12
        # the atomic order gives the same factor to rounding
        sym3, num3, _ = gpu_factor(p, cap, ratio, deterministic=0)
        L3 = num3.export()[2]
        np.testing.assert_allclose(L3, L0, rtol=0, atol=1e-12 * np.abs(L0).max())
    else:
        x, iters, berr = num.solve_refine(b, tol=1e-10)
        x2, iters2, berr2 = num2.solve_refine(b, tol=1e-10)
        assert iters == iters2 and np.array_equal(x.cpu().numpy(), x2.cpu().numpy())


def test_batch_factor_is_bit_identical():
    """A batch of 30 2D Laplacians (thousands of small supernodes sharing
    targets on the lowest levels: the lane-group kernels' scratch and the
    ordered apply) factors to the same bits twice."""
    torch = torch_dev()
    probs = inputs.make_batch(count=30, side_lo=16, side_hi=48)
    mats = [(q.n, q.colptr, q.rowind, q.perm) for q in probs]
    sym = spchol.analyze_batch(mats, sn_cap=150, amalg_ratio=0.2)
    vals_h, rhs_h = inputs.stack_batch(probs)
    vals = torch.from_numpy(vals_h).to("cuda:0")
    b = torch.from_numpy(np.ascontiguousarray(rhs_h)).to("cuda:0")
    num = spchol.factor(sym, vals)
    assert num.status() == 0
    L0, x0 = num.export()[2], num.solve(b).cpu().numpy()
    for _ in range(2):
        num.refactor(vals)
        assert np.array_equal(num.export()[2], L0)
        assert np.array_equal(num.solve(b).cpu().numpy(), x0)


def _dependencies(sym):
    """Edges of the task graph (Section III-A at tile granularity), derived
    from the supernode row lists: F(s) -> T(s, b); T(s, i), T(s, j) ->
    U(s, i, j); U(s, i, j) -> F(t) for each target t of column block j."""
    _, _, sn, _ = sym.export()
    rp, rows = sym.rows()
    ns = len(sn) - 1
    owner = np.repeat(np.arange(ns), np.diff(sn))
    edges = []
    for s in range(ns):
        w = sn[s + 1] - sn[s]
        below = rows[rp[s] + w:rp[s + 1]]
        nb = (len(below) + 63) // 64
        for b in range(nb):
            edges.append(((0, s, 0, 0), (1, s, b, 0)))
        for j in range(nb):
            tg = np.unique(owner[below[64 * j:64 * j + 64]])
            for i in range(j, nb):
                u = (2, s, i, j)
                edges.append(((1, s, i, 0), u))
                edges.append(((1, s, j, 0), u))
                for t in tg:
                    edges.append((u, (0, int(t), 0, 0)))
    return edges


@pytest.mark.parametrize("workers", [1, 2, 0])
def test_task_queue_runs_in_dependency_order(workers):
    """The persistent task-queue kernel with one, two or every resident
    worker (Section IV; Fig. 4's point that a fixed dequeue order must not
    deadlock): its execution log shows every task starting after the tasks
    it depends on finished; with one worker the tasks run one after another
    in ticket order; the factor meets the parity bars."""
    p = inputs.make_grid_problem("lap", (10, 10, 10), 12, sigma=1.0, shift=1e-3, nrhs=0)
    sym, num, _ = gpu_factor(p, 16, 0.1, sched=2, workers=workers, debug_flags=2)
    assert num.status() == 0
    tasks, stamps = num.task_log()
    say("workers", workers, "tasks", len(tasks))
    pos = {}
    for q, (kind, s, a, b) in enumerate(tasks.tolist()):
        pos[(kind, s, a if kind else 0, b if kind == 2 else 0)] = q
    assert (stamps[:, 0] < stamps[:, 1]).all()
    assert len(np.unique(stamps)) == stamps.size  # one clock, every stamp once
    for u, v in _dependencies(sym):
        assert stamps[pos[u], 1] < stamps[pos[v], 0], (u, v)
    if workers == 1:
        assert np.array_equal(stamps.ravel(), np.arange(stamps.size))
    worst, rho, _ = compare_factor(p, num, 16, 0.1, "task queue, %d workers" % workers)
    assert worst <= 1.0 and rho <= 1e-12
