"""GPU checks of batched factorization: many independent SPD matrices of
uneven size through one analysis, one set of factorization launches (level
sets, or the one persistent task-queue launch) and one solve.

The oracle factors the direct sum of the batch (the matrix the batched
analysis defines); bars as for single matrices: FP64 factor entries within
|dL_ij| <= 1e-10 |L_ij| + 1e-13 sqrt(c_ii c_jj) / L_jj, residual <= 1e-12,
every matrix's own backward error <= 1e-14 (FP64 solve) or <= 1e-10 (FP32
factor + FP64 refinement, measured per matrix by the library and by the
oracle); a matrix factored and solved inside the batch matches the same
matrix factored and solved alone to rounding level."""
import numpy as np
import pytest

import oracle
from paper_1608_00044_amd import inputs, spchol
from tests.gpu_util import compare_factor, eta_agreement_atol, say, torch_dev

pytestmark = pytest.mark.gpu


def _batch(count, seed, lo=6, hi=40):
    probs = inputs.make_batch(count=count, seed=seed, side_lo=lo, side_hi=hi)
    probs.append(inputs.random_spd_pattern(90, 0.05, seed=seed, nrhs=1))
    probs.append(inputs.dense_spd(70, seed=seed, nrhs=1))
    return probs


def _factor_batch(probs, sched=0, precision=0, cap=150, ratio=0.1, **extra):
    torch = torch_dev()
    sym = spchol.analyze_batch([(p.n, p.colptr, p.rowind, p.perm) for p in probs], sn_cap=cap,
                               amalg_ratio=ratio, sched=sched, precision=precision, **extra)
    vals, rhs = inputs.stack_batch(probs)
    num = spchol.factor(sym, torch.from_numpy(vals).to("cuda:0"))
    return sym, num, rhs


@pytest.mark.parametrize("sched", [0, 1, 2])
def test_batch_fp64_factor_and_solve(sched):
    torch = torch_dev()
    probs = _batch(12, 77 + sched)
    sym, num, rhs = _factor_batch(probs, sched=sched)
    assert num.status() == 0
    big = inputs.block_diagonal(probs)
    worst, rho, _ = compare_factor(big, num, 150, 0.1, "batch")
    say("batch sched", sched, "n", big.n, "worst/tol", worst, "residual", rho)
    assert worst <= 1.0 and rho <= 1e-12
    x = num.solve(torch.from_numpy(rhs).to("cuda:0")).cpu().numpy().reshape(-1, 1)
    off = 0
    for p in probs:
        xk = x[off:off + p.n]
        eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs, xk)
        assert eta.max() <= 1e-14
        off += p.n


@pytest.mark.parametrize("small", [(-1, 0), (4, 16), (16, 32)])
def test_batch_small_supernode_limits(small):
    """Every split of the supernodes between the lane-group kernels and the
    tile kernels (none small, narrow limits, the default width) factors the
    batch to the same bars."""
    torch = torch_dev()
    probs = _batch(10, 211 + small[0])
    sym, num, rhs = _factor_batch(probs, small_w=small[0], small_r=small[1])
    assert num.status() == 0
    big = inputs.block_diagonal(probs)
    worst, rho, _ = compare_factor(big, num, 150, 0.1, "batch small %s" % (small,))
    say("batch small", small, "worst/tol", worst, "residual", rho)
    assert worst <= 1.0 and rho <= 1e-12
    x = num.solve(torch.from_numpy(rhs).to("cuda:0")).cpu().numpy().reshape(-1, 1)
    off = 0
    for p in probs:
        eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs, x[off:off + p.n])
        assert eta.max() <= 1e-14
        off += p.n
    num.free()
    sym.free()


def test_batch_member_matches_single_factorization():
    torch = torch_dev()
    probs = _batch(9, 5)
    sym, num, rhs = _factor_batch(probs)
    x = num.solve(torch.from_numpy(rhs).to("cuda:0")).cpu().numpy().ravel()
    off = 0
    for k, p in enumerate(probs):
        if k % 3 == 0:
            s1 = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=150, amalg_ratio=0.1)
            n1 = spchol.factor(s1, torch.from_numpy(p.values).to("cuda:0"))
            x1 = n1.solve(torch.from_numpy(np.ascontiguousarray(p.rhs[:, 0])).to("cuda:0"))
            x1 = x1.cpu().numpy()
            np.testing.assert_allclose(x[off:off + p.n], x1, rtol=0,
                                       atol=1e-12 * np.abs(x1).max())
        off += p.n


@pytest.mark.parametrize("sched", [0, 2])
def test_batch_fp32_refined_per_matrix(sched):
    torch = torch_dev()
    probs = _batch(10, 31 + sched)
    sym, num, rhs = _factor_batch(probs, sched=sched, precision=1)
    assert num.status() == 0
    x, iters, berr = num.solve_refine(torch.from_numpy(rhs).to("cuda:0"), tol=1e-10,
                                      max_iter=10)
    assert berr.shape == (len(probs), 1)
    xs = x.cpu().numpy().reshape(-1, 1)
    off = 0
    for k, p in enumerate(probs):
        eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs, xs[off:off + p.n])
        assert eta.max() <= 1e-10
        np.testing.assert_allclose(berr[k, 0], eta[0], rtol=0, atol=eta_agreement_atol(p))
        off += p.n
    say("batch fp32 refine iters", iters, "max eta", berr.max())


@pytest.mark.parametrize("precision", [0, 1])
def test_tuned_batch_options(precision, tmp_path):
    """The autotuner times its candidates through the library on the GPU; the
    options it returns (and caches) factor the batch to the same bars."""
    from paper_1608_00044_amd import tune

    torch = torch_dev()
    probs = inputs.make_batch(count=40, seed=91 + precision, side_lo=6, side_hi=48)
    mats = [(p.n, p.colptr, p.rowind, p.perm) for p in probs]
    vals, rhs = inputs.stack_batch(probs)
    v = torch.from_numpy(vals).to("cuda:0")
    b = torch.from_numpy(np.ascontiguousarray(rhs)).to("cuda:0")
    stages = ((dict(amalg_ratio=0.0), dict(amalg_ratio=0.3)),
              (dict(sn_cap=150), dict(sn_cap=16)),
              (dict(small_w=16, small_r=64), dict(small_w=4, small_r=16),
               dict(small_w=-1, small_r=64)))
    path = str(tmp_path / "tune.json")
    opts, table = tune.tune_batch(mats, v, b, precision, stages, path, steps=1)
    say("tuning", [(t["options"], round(t["ms"], 3), t["nsup"], t["levels"]) for t in table])
    assert len(table) == 5 and all(t["ms"] > 0 for t in table)
    assert table[1]["nsup"] < table[0]["nsup"]  # amalgamation merged supernodes
    assert opts == min(table, key=lambda t: t["ms"])["options"]
    assert tune.tune_batch(mats, v, b, precision, stages, path)[0] == opts
    sym, num, _ = _factor_batch(probs, precision=precision, cap=opts["sn_cap"],
                                ratio=opts["amalg_ratio"], small_w=opts["small_w"],
                                small_r=opts["small_r"])
    assert num.status() == 0
    if precision == 0:
        x = num.solve(b).cpu().numpy()
        bar = 1e-14
    else:
        x, _, _ = num.solve_refine(b, tol=1e-10, max_iter=20)
        x = x.cpu().numpy()
        bar = 1e-10
    off = 0
    for p in probs:
        eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs,
                                    x[off:off + p.n].reshape(-1, 1))
        assert eta.max() <= bar
        off += p.n
    num.free()
    sym.free()
