"""Host-side parts of bench.py: the one-GPU guard, the oracle baselines and
the committed counter summary lookup. No GPU is used."""
import os
import subprocess
import sys

import numpy as np

import bench
from paper_1608_00044_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_batch_members_match_the_whole_batch():
    whole = inputs.make_batch(count=7, side_lo=5, side_hi=12)
    part = inputs.make_batch(count=7, side_lo=5, side_hi=12, members=[5, 2])
    for k, q in zip([5, 2], part):
        p = whole[k]
        assert p.n == q.n
        np.testing.assert_array_equal(p.colptr, q.colptr)
        np.testing.assert_array_equal(p.rowind, q.rowind)
        np.testing.assert_array_equal(p.perm, q.perm)
        np.testing.assert_array_equal(p.values, q.values)
        np.testing.assert_array_equal(p.rhs, q.rhs)


def test_cpu_batch_baseline_small_sample():
    r = bench.cpu_batch_baseline(2000, 6, max_workers=3)
    assert r["kind"] == "oracle" and r["unit"] == "matrices/s"
    assert r["cores"] == 3
    assert r["makespan_s"] <= r["one_core_sum_s"]
    assert r["value"] == 6 / r["pool_wall_s"]  # pool wall time, spawn included
    assert r["makespan_matrices_per_s"] >= r["one_core_matrices_per_s"]
    assert r["factor_flops_F"] > 0


def test_oracle_leg_parity_and_residuals():
    """The oracle leg runs in a thread pinned to one core (the caller's
    affinity is untouched); the parity check passes the oracle's own factor
    and flags a planted error of 1e-8 in one entry; the probe and exact
    residuals of the oracle's factor are at rounding level and see a planted
    1e-6 error."""
    before = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    leg = bench.OracleLeg("lap2d_5pt_64", "lap2d_5pt_64")
    res = leg.join()
    if before is not None:
        assert os.sched_getaffinity(0) == before
    m = res["main"]
    assert m["factor_s"] > 0 and m["flops"] > 0
    n, (Cp, Ci, Cx), Lp, Li, Lx = m["n"], m["C"], m["Lp"], m["Li"], m["Lx"]
    par = bench.factor_parity(n, Cp, Ci, Cx, Lp, Li, Lx, Lp, Li, Lx)
    assert par["structure_contained"] and par["explicit_zeros_ok"]
    assert par["worst_over_tolerance"] == 0.0
    bad = Lx.copy()
    bad[len(bad) // 3] *= 1 + 1e-8
    assert bench.factor_parity(n, Cp, Ci, Cx, Lp, Li, Lx, Lp, Li, bad)["worst_over_tolerance"] > 1
    p = inputs.make_workload("lap2d_5pt_64")
    assert bench.exact_residual(p, Lp, Li, Lx) <= 1e-12
    assert bench.probe_residual(p, Lp, Li, Lx) <= 1e-12
    bad = Lx.copy()
    bad[len(bad) // 2] += 1e-6
    assert bench.exact_residual(p, Lp, Li, bad) > 1e-9
    assert bench.probe_residual(p, Lp, Li, bad) > 1e-9


def test_measured_traffic_follows_the_source():
    assert bench.measured_traffic("k_update", "no_such_workload") is None
    path = os.path.join(ROOT, "profiles", "k_update_traffic_lap3d_7pt_64.txt")
    if os.path.exists(path):
        t = bench.measured_traffic("k_update", "lap3d_7pt_64")
        # present only while the summary's source hash matches the kernel file
        assert t is None or t > 0


def test_hbm_bytes_from_the_structure():
    from paper_1608_00044_amd import spchol

    p = inputs.make_workload("lap2d_5pt_64")
    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=150, amalg_ratio=0.1)
    hb = bench.hbm_bytes(sym)
    _, _, sn, _ = sym.export()
    rp, _ = sym.rows()
    solve = scatter = 0
    for s in range(len(sn) - 1):
        w = int(sn[s + 1] - sn[s])
        r = int(rp[s + 1] - rp[s]) - w
        stored = sum(w - c + r for c in range(w))  # column c stores w - c + r rows
        solve += 2 * (8 * stored + 4 * r)
        scatter += 16 * r * (r + 1) // 2
    assert hb["solve"] == solve and hb["scatter"] == scatter
    assert stored > 0
    sym.free()
