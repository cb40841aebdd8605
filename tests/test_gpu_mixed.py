"""GPU checks of the FP32 factor (FP32 matrix cores, FP32 accumulation) and
of FP64 iterative refinement, against the FP64 oracle, through the C ABI.

Bars: the stored structure holds the exact structure and the explicit zeros
of amalgamated storage stay zero; the FP32 factor's normwise backward error
||L L^T - P A P^T||_F / ||A||_F <= 4 c u (u = 2^-24, c = the largest column
count of L: Cholesky's backward error bound grows with the inner-product
length); the refined solution's normwise backward error (computed by the
oracle) <= 1e-10, and its distance to the oracle's FP64 solution within
4 cond(A) (eta + eta_oracle)."""
import numpy as np
import pytest

import oracle
from paper_1608_00044_amd import inputs, spchol
from tests.gpu_util import eta_agreement_atol, exact_values, say, torch_dev
from tests.test_gpu_parity import _case, _cond_bound

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _fp32_factor(p, cap, ratio, sched=0):
    torch = torch_dev()
    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=cap, amalg_ratio=ratio,
                         sched=sched, precision=1)
    vals = torch.from_numpy(np.ascontiguousarray(p.values)).to("cuda:0")
    num = spchol.factor(sym, vals)
    return sym, num


def _oracle(p):
    Cp, Ci, Cx, _ = oracle.permute(p.n, p.colptr, p.rowind, p.values, p.perm)
    osym = oracle.symbolic(p.n, Cp, Ci)
    st, Lx = oracle.factor(p.n, Cp, Ci, Cx, osym)
    assert st == 0
    return Cp, Ci, Cx, osym, Lx


def _check_refined(p, num, osym, Lx, rhs, tol=1e-10, max_iter=10):
    torch = torch_dev()
    b = torch.from_numpy(np.ascontiguousarray(rhs)).to("cuda:0")
    x, iters, berr = num.solve_refine(b, tol=tol, max_iter=max_iter)
    xs = x.cpu().numpy().reshape(p.n, -1)
    eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, rhs, xs)
    xo = oracle.solve(p.n, osym, Lx, p.perm, rhs).reshape(p.n, -1)
    eta_o = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, rhs, xo)
    kappa = _cond_bound(p)
    fwd = np.abs(xs - xo).max() / np.abs(xo).max()
    say("  refine iters", iters, "eta(lib)", berr.max(), "eta(oracle)", eta.max(),
        "fwd", fwd, "bound", 4 * kappa * (eta.max() + eta_o.max()))
    assert eta.max() <= tol
    assert berr.max() <= tol
    # the library's estimate is the same quantity: the two FP64 residuals
    # differ by their rounding only (eta_agreement_atol), which near
    # convergence can be most of the residual, hence an absolute bar
    np.testing.assert_allclose(berr, eta, rtol=0, atol=eta_agreement_atol(p))
    assert fwd <= max(1e-12, 4 * kappa * (eta.max() + eta_o.max()))
    return iters


MIXED_CASES = ["dense63", "dense150", "dense300", "fig1", "random3", "random4", "lap2d_64",
               "lap2d_40_cap8", "lap3d_20_cap32", "elast27_6", "lap3d_12_shift3"]


def _mixed_case(name):
    if name == "lap3d_12_shift3":
        return inputs.make_grid_problem("lap", (12, 12, 12), 15, sigma=1.0, shift=1e-3,
                                        nrhs=8), 150, 0.1
    return _case(name)


@pytest.mark.parametrize("name,sched", [(c, 0) for c in MIXED_CASES] +
                         [(c, 1) for c in ("dense300", "lap3d_20_cap32", "lap3d_12_shift3")] +
                         [(c, 2) for c in ("dense300", "lap3d_20_cap32", "elast27_6")])
def test_fp32_factor_and_refined_solve(name, sched):
    p, cap, ratio = _mixed_case(name)
    say("case", name, "sched", sched, "n", p.n, "cap", cap, "ratio", ratio)
    sym, num = _fp32_factor(p, cap, ratio, sched)
    assert num.status() == 0
    inf = num.info()
    assert inf["precision"] == 1
    Cp, Ci, Cx, osym, Lx = _oracle(p)
    got, extra = exact_values(num, osym)
    assert (extra == 0.0).all()
    rho = oracle.residual_exact(p.n, Cp, Ci, Cx, osym, got)
    cmax = int(np.diff(osym.Lp).max()) if p.n else 1
    say("  fp32 residual", rho, "bound", 4 * cmax * U32, "fp64 blocks", inf["fp64_blocks"])
    assert rho <= 4 * cmax * U32
    rhs = p.rhs if p.rhs is not None else \
        np.asfortranarray(np.random.default_rng(3).standard_normal((p.n, 2)))
    _check_refined(p, num, osym, Lx, rhs)
    num.free()
    sym.free()


def test_fp64_factor_refines_in_zero_or_one_step():
    p, cap, ratio = _case("lap3d_20_cap32")
    torch = torch_dev()
    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=cap, amalg_ratio=ratio)
    num = spchol.factor(sym, torch.from_numpy(p.values).to("cuda:0"))
    Cp, Ci, Cx, osym, Lx = _oracle(p)
    iters = _check_refined(p, num, osym, Lx, p.rhs, tol=1e-14)
    assert iters <= 2


def test_unstable_pivot_takes_the_fp64_path():
    """A dense SPD matrix whose diagonal block meets a pivot ratio near 2e-5
    (two nearly parallel rows): the FP32 pass flags the block, it is factored
    again in FP64, and refinement still reaches 1e-10; a well-conditioned
    matrix of the same shape takes no FP64 block."""
    torch = torch_dev()
    n, eps = 40, 1e-5
    rng = np.random.default_rng(11)
    a = np.eye(n) * 2.0
    a[0, 1] = a[1, 0] = 2.0 * (1.0 - eps)
    a += 1e-6 * (lambda g: g @ g.T)(rng.standard_normal((n, n))) / n  # pivot 2 ~ 4e-5
    j, i = np.meshgrid(np.arange(n), np.arange(n))
    m = i >= j
    cp, ri, vx = inputs.lower_csc_from_coo(n, i[m], j[m], a[m])
    rhs = np.asfortranarray(rng.standard_normal((n, 2)))
    p = inputs.Problem(n, cp, ri.astype(np.int32), vx, None, rhs)
    sym, num = _fp32_factor(p, 150, 0.0)
    assert num.status() == 0
    assert num.info()["fp64_blocks"] == 1
    Cp, Ci, Cx, osym, Lx = _oracle(p)
    x, iters, berr = num.solve_refine(torch.from_numpy(rhs).to("cuda:0"), tol=1e-10, max_iter=20)
    eta = oracle.backward_error(n, cp, ri, vx, rhs, x.cpu().numpy())
    assert eta.max() <= 1e-10
    q = inputs.dense_spd(n, seed=5, nrhs=0)
    sym2, num2 = _fp32_factor(q, 150, 0.0)
    assert num2.status() == 0 and num2.info()["fp64_blocks"] == 0


@pytest.mark.parametrize("k", [1, 37, 300])
def test_fp32_non_spd_reports_first_failing_column(k):
    n = 400
    p = inputs.tridiag(n)
    vals = p.values.copy()
    vals[p.colptr[k - 1]] = (k - 1) / k - 0.5
    sym, num = _fp32_factor(inputs.Problem(n, p.colptr, p.rowind, vals, None), 150, 0.0)
    assert num.status() == k
    torch = torch_dev()
    with pytest.raises(spchol.SpcError) as e:
        num.solve_refine(torch.ones(n, dtype=torch.float64, device="cuda:0"))
    assert e.value.status == k


def test_refine_reports_not_converged_and_checks_arguments():
    torch = torch_dev()
    p, cap, ratio = _mixed_case("lap3d_12_shift3")
    sym, num = _fp32_factor(p, cap, ratio)
    b = torch.from_numpy(np.ascontiguousarray(p.rhs[:, :1])).to("cuda:0")
    x, iters, berr = num.solve_refine(b, tol=1e-30, max_iter=2, check=False)
    assert num.last_refine_status == spchol.SPC_ERR_NOT_CONVERGED and iters == 2
    assert berr[0] > 1e-30
    with pytest.raises(spchol.SpcError) as e:
        num.solve_refine(b, x=b)  # b and x must not overlap
    assert e.value.status == spchol.SPC_ERR_ARG
    with pytest.raises(spchol.SpcError) as e:
        num.solve_refine(b, tol=-1.0)
    assert e.value.status == spchol.SPC_ERR_ARG


def test_fp32_plain_solve_and_refactor():
    """spc_solve on an FP32 factor is an FP32 solve (backward error near u32);
    a refactorization with new values refines to 1e-10 again."""
    torch = torch_dev()
    p = inputs.make_grid_problem("27pt3", (7, 7, 7), 41, shift=1e-3, nrhs=3)
    sym, num = _fp32_factor(p, 150, 0.1)
    b = torch.from_numpy(np.ascontiguousarray(p.rhs)).to("cuda:0")
    x = num.solve(b).cpu().numpy()
    eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs, x)
    assert eta.max() <= 1e-5
    p2 = inputs.make_grid_problem("27pt3", (7, 7, 7), 42, shift=1e-3, nrhs=3)
    num.refactor(torch.from_numpy(p2.values).to("cuda:0"))
    assert num.status() == 0
    Cp, Ci, Cx, osym, Lx = _oracle(p2)
    _check_refined(p2, num, osym, Lx, p2.rhs)


@pytest.mark.parametrize("k", [1, 8, 11])
def test_refine_right_hand_side_groups(k):
    """The residual goes through A eight right-hand sides at a time: one, a
    full group and a ragged second group all refine to 1e-10, and the last
    column agrees with its own one-column refinement to within the bound two
    backward-stable solutions share."""
    torch = torch_dev()
    p = inputs.make_grid_problem("27pt3", (6, 6, 6), 43, shift=1e-3, nrhs=0)
    sym, num = _fp32_factor(p, 150, 0.1)
    Cp, Ci, Cx, osym, Lx = _oracle(p)
    B = np.asfortranarray(np.random.default_rng(k).standard_normal((p.n, k)))
    _check_refined(p, num, osym, Lx, B)
    b = torch.from_numpy(B).to("cuda:0")
    x, _, _ = num.solve_refine(b, tol=1e-10)
    x = x.cpu().numpy().reshape(p.n, k)
    xl, _, _ = num.solve_refine(torch.from_numpy(np.ascontiguousarray(B[:, k - 1])).to("cuda:0"),
                                tol=1e-10)
    xl = xl.cpu().numpy().reshape(p.n)
    # both meet eta <= 1e-10, so they agree to within cond(A) times twice that
    bound = max(1e-12, 4 * _cond_bound(p) * 2e-10)
    assert np.abs(x[:, k - 1] - xl).max() / np.abs(xl).max() <= bound


def test_refinement_stall_switches_to_fp64_factor():
    """A 2D Laplacian with a 1e-8 shift has cond(A) near 8e8, so FP32
    corrections (u32 cond(A) ~ 50) cannot converge: after two steps in which
    the worst eta does not halve, the corrections continue with an FP64
    factor of the same matrix and reach 1e-10 (checked by the oracle's
    definition); a refactorization makes the FP64 factor again.  A
    well-conditioned problem never needs it."""
    torch = torch_dev()
    p = inputs.make_grid_problem("lap", (48, 48), 71, sigma=None, shift=1e-8, nrhs=2)
    sym, num = _fp32_factor(p, 150, 0.0)
    assert num.status() == 0
    b = torch.from_numpy(np.ascontiguousarray(p.rhs)).to("cuda:0")
    x, iters, berr = num.solve_refine(b, tol=1e-10, max_iter=30)
    eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs,
                                x.cpu().numpy().reshape(p.n, -1))
    say("stalled refinement: iters", iters, "eta", eta.max(), "info", num.info())
    assert eta.max() <= 1e-10 and berr.max() <= 1e-10
    assert num.info()["refine_fallbacks"] == 1
    num.refactor(torch.from_numpy(p.values).to("cuda:0"))
    x2, _, _ = num.solve_refine(b, tol=1e-10, max_iter=30)
    assert num.info()["refine_fallbacks"] == 2
    eta2 = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs,
                                 x2.cpu().numpy().reshape(p.n, -1))
    assert eta2.max() <= 1e-10
    q = inputs.make_grid_problem("27pt3", (6, 6, 6), 43, shift=1e-3, nrhs=1)
    sym2, num2 = _fp32_factor(q, 150, 0.1)
    num2.solve_refine(torch.from_numpy(np.ascontiguousarray(q.rhs)).to("cuda:0"), tol=1e-10)
    assert num2.info()["refine_fallbacks"] == 0
