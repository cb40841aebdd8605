"""GPU checks of the solves' persistent launch over the top levels of the
supernodal elimination tree (spc_options.solve_tail in the atomic
contribution order, the dependency counters of Section IV applied to the two
solves of Section II-A): the solution is backward stable, agrees with the
level-by-level sweeps to rounding, run after run, and holds for ragged
right-hand-side groups, the FP32 factor under refinement, a batch with
several roots in the tail, and the allocation-free entry point."""
import numpy as np
import pytest

import oracle
from paper_1608_00044_amd import inputs, spchol
from tests.gpu_util import gpu_factor, say, torch_dev

pytestmark = pytest.mark.gpu


def _problem(name, nrhs):
    if name == "lap3d_24":
        return inputs.make_grid_problem("lap", (24, 24, 24), 8, sigma=1.0, shift=1e-6,
                                        nrhs=nrhs), 150, 0.1, {}
    if name == "lap3d_20_cap32":
        return inputs.make_grid_problem("lap", (20, 20, 20), 6, sigma=1.0, shift=1e-6,
                                        nrhs=nrhs), 32, 0.1, {}
    if name == "elast27_8":
        return inputs.make_grid_problem("27pt3", (8, 8, 8), 10, shift=1e-3,
                                        nrhs=nrhs), 150, 0.1, {}
    if name == "lap3d_16_cap16":
        # every supernode on the workgroup kernels: a tail of 114 levels of
        # at most 16 columns
        return inputs.make_grid_problem("lap", (16, 16, 16), 3, sigma=1.0, shift=1e-6,
                                        nrhs=nrhs), 16, 0.0, {"small_w": -1}
    raise KeyError(name)


def _solve(num, b):
    return num.solve(b if b.shape[1] > 1 else b[:, 0]).cpu().numpy().reshape(b.shape[0], -1)


@pytest.mark.parametrize("name,nrhs", [("lap3d_24", 1), ("lap3d_24", 3), ("lap3d_24", 20),
                                       ("lap3d_20_cap32", 1), ("elast27_8", 2),
                                       ("lap3d_16_cap16", 9)])
def test_tail_solve_matches_level_sweeps(name, nrhs):
    """Solutions through the tail and level by level (the default); the
    deterministic order has no tail."""
    torch = torch_dev()
    p, cap, ratio, opts = _problem(name, nrhs)
    sym, num, vals = gpu_factor(p, cap, ratio, deterministic=0, solve_tail=1, **opts)
    info = sym.info()
    say("case", name, "nrhs", nrhs, "n", p.n, "levels", info["nlevels"], "tail levels",
        info["tail_levels"], "tail supernodes", info["tail_supernodes"])
    assert info["tail_levels"] >= 2
    assert num.status() == 0
    symD = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=cap, amalg_ratio=ratio,
                          solve_tail=1, **opts)
    assert symD.info()["tail_levels"] == 0
    symD.free()
    symL, numL, _ = gpu_factor(p, cap, ratio, deterministic=0, **opts)
    assert symL.info()["tail_levels"] == 0
    b = torch.from_numpy(np.ascontiguousarray(p.rhs)).to("cuda:0")
    x = _solve(num, b)
    xl = _solve(numL, b)
    eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs, x)
    eta_l = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs, xl)
    diff = np.abs(x - xl).max() / np.abs(xl).max()
    say("  backward error", eta.max(), "level sweeps", eta_l.max(), "difference", diff)
    assert eta.max() <= 1e-14
    # same factor, two summation orders of the same solves: rounding apart
    assert diff <= 1e-9
    for rep in range(3):
        torch.randn(4096, device="cuda:0").sum().item()
        xr = _solve(num, b)
        assert np.abs(xr - x).max() <= 1e-9 * np.abs(x).max(), "repeat %d" % rep
    for o in (num, numL, sym, symL):
        o.free()


def test_tail_solve_fp32_refinement():
    torch = torch_dev()
    p, cap, ratio, _ = _problem("elast27_8", 8)
    sym, num, _ = gpu_factor(p, cap, ratio, precision=1, deterministic=0, solve_tail=1)
    assert sym.info()["tail_levels"] >= 2 and num.status() == 0
    b = torch.from_numpy(np.ascontiguousarray(p.rhs)).to("cuda:0")
    x, iters, berr = num.solve_refine(b, tol=1e-10)
    eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs, x.cpu().numpy())
    say("refined: iterations", iters, "backward error", eta.max())
    assert eta.max() <= 1e-10
    x2, iters2, berr2 = num.solve_refine(b, tol=1e-10)
    assert np.asarray(berr2).max() <= 1e-10


def test_tail_solve_batch_with_several_roots():
    """A batch whose tallest members reach the tail levels on their own: the
    tail holds several roots (each with no backward block before it)."""
    torch = torch_dev()
    probs = inputs.make_batch(count=12, side_lo=40, side_hi=90, seed=5)
    mats = [(q.n, q.colptr, q.rowind, q.perm) for q in probs]
    vals_h, rhs_h = inputs.stack_batch(probs)
    vals = torch.from_numpy(vals_h).to("cuda:0")
    b = torch.from_numpy(np.ascontiguousarray(rhs_h)).to("cuda:0")
    out = []
    for tail in (1, 0):
        sym = spchol.analyze_batch(mats, sn_cap=150, amalg_ratio=0.2, small_w=-1,
                                   deterministic=0, solve_tail=tail)
        say("tail option", tail, "levels", sym.info()["nlevels"], "tail levels",
            sym.info()["tail_levels"])
        num = spchol.factor(sym, vals)
        assert num.status() == 0
        out.append(num.solve(b).cpu().numpy())
        num.free()
        sym.free()
    assert np.abs(out[0] - out[1]).max() <= 1e-9 * np.abs(out[1]).max()
    off = 0
    for q in probs:
        xq = out[0][off:off + q.n]
        eta = oracle.backward_error(q.n, q.colptr, q.rowind, q.values, q.rhs, xq.reshape(q.n, -1))
        assert eta.max() <= 1e-14
        off += q.n


def test_tail_solve_noalloc_matches():
    torch = torch_dev()
    p, cap, ratio, _ = _problem("lap3d_24", 2)
    sym, num, _ = gpu_factor(p, cap, ratio, deterministic=0, solve_tail=1)
    assert sym.info()["tail_levels"] >= 2
    # column-major operands, as the allocation-free entry point takes them
    b = torch.from_numpy(np.asfortranarray(p.rhs)).to("cuda:0").t().contiguous().t()
    x = num.solve(b).cpu().numpy()
    x2 = torch.full((b.shape[1], p.n), np.nan, dtype=torch.float64, device="cuda:0").t()
    got = num.solve_noalloc(b, x2).cpu().numpy()
    assert np.abs(got - x).max() <= 1e-9 * np.abs(x).max()
