"""GPU check of spc_solve_noalloc, the solve for callers that cannot allocate
device memory (its work lives in one static 64 MiB device array): through
the C ABI it gives the same bits as spc_solve on the same factor, on two
calls in a row, the second with a smaller input (a smaller matrix and fewer
right-hand sides, so the array keeps the first call's contents), in FP64 and
FP32; work beyond the array is refused before any device work."""
import numpy as np
import pytest

from paper_1608_00044_amd import inputs, spchol
from tests.gpu_util import gpu_factor, say, torch_dev

pytestmark = pytest.mark.gpu


def _solve_both(p, cap, ratio, nrhs, precision=0):
    torch = torch_dev()
    sym, num, _ = gpu_factor(p, cap, ratio, precision=precision)
    assert num.status() == 0
    B = np.asfortranarray(np.random.default_rng(nrhs).standard_normal((p.n, nrhs)))
    b = torch.from_numpy(B).to("cuda:0").t().contiguous().t()
    want = num.solve(b).cpu().numpy()
    x = torch.full((nrhs, p.n), np.nan, dtype=torch.float64, device="cuda:0").t()
    got = num.solve_noalloc(b, x).cpu().numpy()
    say("n", p.n, "nrhs", nrhs, "precision", precision, "max |diff|",
        np.abs(got - want).max())
    assert np.array_equal(got, want)
    num.free()
    sym.free()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_solve_matches_solve_twice(precision):
    big = inputs.make_grid_problem("lap", (20, 20, 20), 81, sigma=1.0, shift=1e-3, nrhs=0)
    small = inputs.make_grid_problem("lap", (9, 9, 9), 82, sigma=1.0, shift=1e-3, nrhs=0)
    _solve_both(big, 150, 0.1, 11, precision)
    _solve_both(small, 150, 0.1, 2, precision)


def test_noalloc_solve_refuses_work_beyond_the_array():
    torch = torch_dev()
    p = inputs.make_grid_problem("lap", (8, 8, 8), 83, sigma=1.0, shift=1e-3, nrhs=0)
    sym, num, _ = gpu_factor(p, 150, 0.1)
    per_rhs = sym.info()["solve_bytes_per_rhs"]
    k = (64 << 20) // per_rhs + 1  # one column more than fits
    b = torch.ones((k, p.n), dtype=torch.float64, device="cuda:0").t()
    x = torch.zeros((k, p.n), dtype=torch.float64, device="cuda:0").t()
    with pytest.raises(spchol.SpcError) as e:
        num.solve_noalloc(b, x)
    assert e.value.status == spchol.SPC_ERR_TOO_LARGE
    assert float(x.abs().max()) == 0.0  # untouched
    # the largest count that fits is solved
    k2 = (64 << 20) // per_rhs
    got = num.solve_noalloc(b[:, :k2], x[:, :k2]).cpu().numpy()
    want = num.solve(b[:, :k2].contiguous()).cpu().numpy()
    assert np.array_equal(got, want)
