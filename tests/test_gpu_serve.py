"""GPU checks of the request server: continuous batching of factor+solve and
solve-only requests over resident patterns.

Bars: every result of a mix run with overlapping requests (several on the
device at once) equals the same request run alone bit for bit (the
deterministic order of every sum in factor and solve), and is backward
stable against the oracle's definition (<= 1e-14); admission keeps
the resident bytes within the budget, evicting idle factors; a request whose
pattern cannot fit, a solve-only request with no factor, and a failed pivot
are reported per request."""
import numpy as np
import pytest

import oracle
from paper_1608_00044_amd import inputs, spchol
from tests.gpu_util import say, torch_dev

pytestmark = pytest.mark.gpu


def _patterns():
    probs = [inputs.make_grid_problem("lap", (20, 20), 61, sigma=1.0, shift=1e-3, nrhs=0),
             inputs.make_grid_problem("lap", (33, 33), 62, sigma=1.0, shift=1e-3, nrhs=0),
             inputs.make_grid_problem("lap", (8, 8, 8), 63, sigma=1.0, shift=1e-3, nrhs=0),
             inputs.make_grid_problem("lap", (11, 11, 11), 64, sigma=1.0, shift=1e-3, nrhs=0),
             inputs.dense_spd(60, seed=65, nrhs=0)]
    syms = [spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=150, amalg_ratio=0.1)
            for p in probs]
    return probs, syms


def _requests(probs, count, seed):
    """Seeded mix: each pattern starts with a factor request; then 30% solve-only."""
    rng = np.random.default_rng(seed)
    reqs = [(k, 0, 4) for k in range(len(probs))]
    for _ in range(count - len(probs)):
        reqs.append((int(rng.integers(len(probs))), int(rng.random() < 0.3),
                     int(rng.choice([1, 4, 16, 64]))))
    return reqs


def _run(server_opts, probs, syms, reqs, sequential, seed=7):
    torch = torch_dev()
    torch.zeros(1, device="cuda:0")
    srv = spchol.Server(**server_opts)
    pids = [srv.add_pattern(s) for s in syms]
    vals = [torch.from_numpy(p.values).to("cuda:0") for p in probs]
    rng = np.random.default_rng(seed)
    Bs = [np.asfortranarray(rng.standard_normal((probs[k].n, nr))) for k, _, nr in reqs]
    out = []
    tickets = []
    for (k, kind, nr), B in zip(reqs, Bs):
        b = torch.from_numpy(B).to("cuda:0").t().contiguous().t()
        x = torch.zeros((nr, probs[k].n), dtype=torch.float64, device="cuda:0").t()
        t = srv.submit(pids[k], b, x, values=vals[k] if kind == 0 else None)
        tickets.append((t, x))
        if sequential:
            out.append((srv.wait(t), x.cpu().numpy()))
    if not sequential:
        out = [(srv.wait(t), x.cpu().numpy()) for t, x in tickets]
    stats = srv.stats()
    srv.destroy()
    return out, Bs, stats


def test_mix_matches_alone_and_overlaps():
    probs, syms = _patterns()
    reqs = _requests(probs, 48, 5)
    alone, Bs, st1 = _run(dict(max_inflight=1), probs, syms, reqs, sequential=True)
    mix, _, st2 = _run(dict(max_inflight=8), probs, syms, reqs, sequential=False)
    say("alone peak inflight", st1["peak_inflight"], "mix peak inflight", st2["peak_inflight"],
        "resident", st2["resident_factors"], "peak MB", st2["peak_bytes"] / 2 ** 20)
    assert st1["peak_inflight"] == 1 and st2["peak_inflight"] > 1
    lat = []
    for (k, kind, nr), (ra, xa), (rm, xm), B in zip(reqs, alone, mix, Bs):
        p = probs[k]
        assert ra["status"] == 0 and rm["status"] == 0
        assert np.array_equal(xm, xa)
        eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, B, xm)
        assert eta.max() <= 1e-14
        lat.append(rm["latency_ms"])
    say("mix latency p50 %.3f p99 %.3f ms" % (np.percentile(lat, 50), np.percentile(lat, 99)))


def test_admission_within_budget_evicts_idle_factors():
    torch = torch_dev()
    probs, syms = _patterns()
    # a factor with its work vectors for 4 columns; every pattern's device plan
    # is charged once, with its first factor, and stays until the handle is
    # freed: the budget holds every plan and one and a half factors
    per = [s.info()["factor_bytes"] + 4 * s.info()["solve_bytes_per_rhs"] for s in syms]
    plans = sum(s.info()["plan_bytes"] for s in syms)
    budget = plans + max(per) + min(per) // 2
    reqs = [(k % len(probs), 0, 4) for k in range(3 * len(probs))]
    out, Bs, st = _run(dict(max_inflight=4, max_nrhs=4, mem_budget_bytes=budget), probs, syms,
                       reqs, sequential=False)
    say("budget", budget, "peak", st["peak_bytes"], "evictions", st["evictions"])
    assert all(r["status"] == 0 for r, _ in out)
    assert st["peak_bytes"] <= budget and st["evictions"] > 0
    for (k, _, _), (r, x), B in zip(reqs, out, Bs):
        p = probs[k]
        assert oracle.backward_error(p.n, p.colptr, p.rowind, p.values, B, x).max() <= 1e-14
    # a pattern larger than the whole budget is refused per request
    srv = spchol.Server(max_inflight=2, max_nrhs=4, mem_budget_bytes=min(per) // 2)
    pid = srv.add_pattern(syms[0])
    b = torch.ones((probs[0].n, 1), dtype=torch.float64, device="cuda:0")
    x = torch.zeros_like(b)
    t = srv.submit(pid, b, x, values=torch.from_numpy(probs[0].values).to("cuda:0"))
    assert srv.wait(t)["status"] == spchol.SPC_ERR_OOM
    srv.destroy()


def test_solve_only_statuses_and_failed_factor_keeps_previous():
    torch = torch_dev()
    n = 300
    p = inputs.tridiag(n)
    sym = spchol.analyze(p.n, p.colptr, p.rowind)
    srv = spchol.Server(max_inflight=4, max_nrhs=2)
    pid = srv.add_pattern(sym)
    b = torch.from_numpy(np.ones((n, 1))).to("cuda:0")
    x = torch.zeros_like(b)
    assert srv.wait(srv.submit(pid, b, x))["status"] == spchol.SPC_ERR_NOT_FACTORED
    good = torch.from_numpy(p.values).to("cuda:0")
    assert srv.wait(srv.submit(pid, b, x, values=good))["status"] == 0
    bad_v = p.values.copy()
    bad_v[p.colptr[44]] = 44 / 45 - 0.5
    bad = torch.from_numpy(bad_v).to("cuda:0")
    x2 = torch.zeros_like(b)
    assert srv.wait(srv.submit(pid, b, x2, values=bad))["status"] == 45
    x3 = torch.zeros_like(b)
    assert srv.wait(srv.submit(pid, b, x3))["status"] == 0  # the good factor is still current
    with pytest.raises(spchol.SpcError) as busy:  # the server holds the pattern
        sym.free()
    assert busy.value.status == spchol.SPC_ERR_BUSY
    eta = oracle.backward_error(n, p.colptr, p.rowind, p.values, np.ones((n, 1)), x3.cpu().numpy())
    assert eta.max() <= 1e-14
    with pytest.raises(spchol.SpcError):
        srv.submit(pid, torch.ones((3, n), dtype=torch.float64, device="cuda:0").t(),
                   torch.zeros((3, n), dtype=torch.float64, device="cuda:0").t())  # nrhs > 2
    with pytest.raises(ValueError):  # values of the wrong length
        srv.submit(pid, b, x, values=good[:-1])
    srv.destroy()
    sym.free()  # released by the server
