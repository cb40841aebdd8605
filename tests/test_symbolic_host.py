"""Host logic of the HIP library, on the CPU: the C ABI loads and exports every
declared symbol, argument checks, and the symbolic analysis matches the
oracle's bit for bit."""
import dataclasses
import os
import re

import numpy as np
import pytest

import oracle
from paper_1608_00044_amd import inputs, spchol
from tests.helpers import load_fig1, refusal_case, spd_values_for_pattern

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "spchol.h")).read()
    declared = set(re.findall(r"\b(spc_[a-z_]+)\s*\(", hdr))
    assert declared == set(spchol.EXPORTS)
    L = spchol.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_status_strings():
    assert spchol.status_string(0) == "success"
    assert "pivot" in spchol.status_string(7)
    assert spchol.status_string(spchol.SPC_ERR_PATTERN).startswith("malformed")


@pytest.mark.parametrize("rows,code", [([1, 0, 1, 2, 3], spchol.SPC_ERR_PATTERN),
                                       ([0, 0, 1, 2, 3], spchol.SPC_ERR_PATTERN),
                                       ([0, 1, 0, 2, 3], spchol.SPC_ERR_PATTERN),
                                       ([0, 1, 1, 2, 4], spchol.SPC_ERR_PATTERN)])
def test_analyze_rejects_bad_patterns(rows, code):
    with pytest.raises(spchol.SpcError) as e:
        spchol.analyze(4, [0, 2, 3, 4, 5], rows)
    assert e.value.status == code


def test_analyze_rejects_bad_arguments():
    cp, ri = [0, 1, 2], [0, 1]
    with pytest.raises(spchol.SpcError) as e:
        spchol.analyze(2, cp, ri, perm=[0, 0])
    assert e.value.status == spchol.SPC_ERR_ARG
    for kw in (dict(sn_cap=0), dict(sn_cap=151), dict(amalg_ratio=-0.1), dict(sched=3), dict(sched=-1),
               dict(mem_budget_bytes=-1), dict(spin_limit=-1), dict(precision=2),
               dict(precision=-1), dict(threads=-1), dict(small_w=17), dict(small_w=-2),
               dict(small_r=65), dict(small_r=-1)):
        with pytest.raises(spchol.SpcError) as e:
            spchol.analyze(2, cp, ri, **kw)
        assert e.value.status == spchol.SPC_ERR_ARG
    for kw in (dict(small_w=-1), dict(small_w=1, small_r=1), dict(small_w=16, small_r=64)):
        spchol.analyze(2, cp, ri, **kw).free()


def _compare_with_oracle(p, cap=150, ratio=0.0):
    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=cap, amalg_ratio=ratio)
    parent, cc, sn, snp = sym.export()
    Cp, Ci, Cx, _ = oracle.permute(p.n, p.colptr, p.rowind, p.values, p.perm)
    osym = oracle.symbolic(p.n, Cp, Ci)
    assert np.array_equal(parent, osym.parent)
    assert np.array_equal(cc, osym.colcount)
    osn = oracle.supernode_partition(p.n, osym.parent, osym.colcount, cap, ratio)
    assert np.array_equal(sn, osn)
    assert np.array_equal(snp, oracle.supernodal_parent(osym.parent, osn))
    inf = sym.info()
    assert inf["nnz_l"] == osym.nnz
    assert inf["flops"] == float(osym.flops)
    # stored rows below each supernode = exact structure of its last column
    rp, rows = sym.rowptr_rows = sym.rows()
    for s in range(len(sn) - 1):
        a, b = sn[s], sn[s + 1] - 1
        got = rows[rp[s]:rp[s + 1]]
        assert got[: b - a + 1].tolist() == list(range(a, b + 1))
        assert np.array_equal(got[b - a + 1:], osym.Li[osym.Lp[b] + 1:osym.Lp[b + 1]])
    return sym, osym, sn


def _check_relative_indices(sym, sn):
    rp, rows = sym.rows()
    pr = sym.pairs()
    ns = len(sn) - 1
    owner = np.repeat(np.arange(ns), np.diff(sn))
    cover = {}
    for p in range(len(pr["src"])):
        s, t = int(pr["src"][p]), int(pr["tgt"][p])
        b, e = pr["seg"][p]
        w = sn[s + 1] - sn[s]
        below = rows[rp[s] + w:rp[s + 1]]
        assert t > s
        # the segment holds exactly the source rows inside t's columns
        assert (owner[below[b:e]] == t).all()
        assert b == 0 or owner[below[b - 1]] < t
        assert e == len(below) or owner[below[e]] > t
        # relative index invariant: rows_t[rel[i]] == rows_s[i] for every i >= b
        rt = rows[rp[t]:rp[t + 1]]
        rel = pr["rel"][pr["rel_off"][p]:pr["rel_off"][p] + len(below) - b]
        assert np.array_equal(rt[rel], below[b:])
        cover.setdefault(s, []).append((b, e))
    for s in range(ns):
        w = sn[s + 1] - sn[s]
        r = rp[s + 1] - rp[s] - w
        segs = sorted(cover.get(s, []))
        pos = 0
        for b, e in segs:
            assert b == pos
            pos = e
        assert pos == r


def test_fig1_bit_exact():
    fig = load_fig1()
    p = spd_values_for_pattern(fig["n"], fig["orig"], seed=1)
    sym, osym, sn = _compare_with_oracle(p)
    assert len(sn) - 1 == 10
    _check_relative_indices(sym, sn)


@pytest.mark.parametrize("seed", range(30))
def test_random_bit_exact(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    p = inputs.random_spd_pattern(n, float(rng.uniform(0.02, 0.3)), seed=seed)
    cap = int(rng.choice([1, 2, 3, 8, 150]))
    ratio = float(rng.choice([0.0, 0.1, 0.5]))
    sym, _, sn = _compare_with_oracle(p, cap, ratio)
    _check_relative_indices(sym, sn)


@pytest.mark.parametrize("dims,cap,ratio", [((64, 64), 150, 0.0), ((12, 12, 12), 150, 0.1),
                                            ((20, 20, 20), 32, 0.1), ((40, 40), 150, 0.3)])
def test_grid_bit_exact(dims, cap, ratio):
    p = inputs.make_grid_problem("lap", dims, seed=7, sigma=1.0, shift=1e-6, nrhs=0)
    sym, _, sn = _compare_with_oracle(p, cap, ratio)
    if p.n <= 5000:
        _check_relative_indices(sym, sn)


def test_cfg2_symbolic_bit_exact():
    """Full-size 64^3 7-point workload with amalgamation 0.1 (integer parity)."""
    p = inputs.make_workload("lap3d_7pt_64", nrhs=0)
    _compare_with_oracle(p, 150, 0.1)


def test_empty_and_single():
    sym = spchol.analyze(0, [0], [])
    assert sym.info()["nsup"] == 0
    sym = spchol.analyze(1, [0, 1], [0])
    parent, cc, sn, snp = sym.export()
    assert parent.tolist() == [-1] and cc.tolist() == [1] and sn.tolist() == [0, 1]


def test_missing_diagonal_is_structural():
    # column 1 has no diagonal entry: still analyzable (its pivot will be zero)
    sym = spchol.analyze(3, [0, 2, 2, 3], [0, 1, 2])
    parent, cc, _, _ = sym.export()
    assert parent.tolist() == [1, -1, -1]


def _check_task_order(sym, sn, workers):
    """The task-queue order is a topological order of the F/T/U task graph and
    the F counters count (tile, distinct target) pairs; derived here from the
    supernode row lists alone."""
    tk, cnt0 = sym.tasks(workers)
    rp, rows = sym.rows()
    ns = len(sn) - 1
    owner = np.repeat(np.arange(ns), np.diff(sn))
    pos = {}
    for q, (kind, s, a, b) in enumerate(tk.tolist()):
        key = (kind, s, a, b) if kind == 2 else ((kind, s, a) if kind == 1 else (kind, s))
        assert key not in pos
        pos[key] = q
    expect_cnt = np.zeros(ns, dtype=np.int64)
    want = 0
    for s in range(ns):
        w = sn[s + 1] - sn[s]
        below = rows[rp[s] + w:rp[s + 1]]
        nb = (len(below) + 63) // 64
        want += 1 + nb + nb * (nb + 1) // 2
        for b in range(nb):
            assert pos[(0, s)] < pos[(1, s, b)]
        for j in range(nb):
            tg = np.unique(owner[below[64 * j:64 * j + 64]])
            for i in range(j, nb):
                u = pos[(2, s, i, j)]
                assert pos[(1, s, i)] < u and pos[(1, s, j)] < u
                for t in tg:
                    assert u < pos[(0, int(t))]
                    expect_cnt[t] += 1
    assert len(tk) == want
    assert np.array_equal(cnt0, expect_cnt)


@pytest.mark.parametrize("case", ["fig1", "rand0", "rand1", "grid12", "grid2d"])
@pytest.mark.parametrize("workers", [1, 7, 256])
def test_task_order_is_topological(case, workers):
    if case == "fig1":
        fig = load_fig1()
        p = spd_values_for_pattern(fig["n"], fig["orig"], seed=1)
        cap, ratio = 150, 0.0
    elif case.startswith("rand"):
        p = inputs.random_spd_pattern(150, 0.1, seed=int(case[-1]))
        cap, ratio = 8, 0.1
    elif case == "grid12":
        p = inputs.make_grid_problem("lap", (12, 12, 12), seed=3, sigma=1.0, shift=1e-3, nrhs=0)
        cap, ratio = 150, 0.1
    else:
        p = inputs.make_grid_problem("lap", (90, 90), seed=3, sigma=1.0, shift=1e-3, nrhs=0)
        cap, ratio = 32, 0.0
    sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=cap, amalg_ratio=ratio, sched=2)
    _, _, sn, _ = sym.export()
    _check_task_order(sym, sn, workers)


def test_task_order_arguments():
    sym = spchol.analyze(1, [0, 1], [0], sched=2)
    with pytest.raises(spchol.SpcError) as e:
        sym.tasks(0)
    assert e.value.status == spchol.SPC_ERR_ARG
    tk, cnt0 = sym.tasks(4)
    assert tk.tolist() == [[0, 0, 0, 0]] and cnt0.tolist() == [0]


def test_batch_analysis_is_the_union_of_single_analyses():
    """The batched analysis of independent matrices equals their single
    analyses side by side: etree, column counts, supernodes (never across two
    matrices) and row lists, shifted by each matrix's offset."""
    probs = inputs.make_batch(count=6, side_lo=5, side_hi=17)
    probs.append(inputs.random_spd_pattern(40, 0.1, seed=3))
    probs.append(inputs.tridiag(1))
    mats = [(p.n, p.colptr, p.rowind, p.perm) for p in probs]
    bs = spchol.analyze_batch(mats, sn_cap=16, amalg_ratio=0.1)
    inf = bs.info()
    assert inf["nbatch"] == len(probs) and inf["n"] == sum(p.n for p in probs)
    parent, cc, sn, _ = bs.export()
    rp, rows = bs.rows()
    off, s_at = 0, 0
    flops = 0.0
    for p in probs:
        one = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, sn_cap=16, amalg_ratio=0.1)
        par1, cc1, sn1, _ = one.export()
        rp1, rows1 = one.rows()
        assert np.array_equal(parent[off:off + p.n], np.where(par1 < 0, -1, par1 + off))
        assert np.array_equal(cc[off:off + p.n], cc1)
        ns1 = len(sn1) - 1
        assert np.array_equal(sn[s_at:s_at + ns1 + 1], sn1 + off)
        got = rows[rp[s_at]:rp[s_at + ns1]]
        assert np.array_equal(got, rows1 + off)
        flops += one.info()["flops"]
        off += p.n
        s_at += ns1
    assert s_at == inf["nsup"] and inf["flops"] == flops


def _whole_analysis_fields(sym):
    inf = sym.info()
    inf.pop("nbatch")
    out = {"info": inf}
    out["parent"], out["cc"], out["sn"], out["snpar"] = sym.export()
    out["rowptr"], out["rows"] = sym.rows()
    for k, v in sym.pairs().items():
        out["pair_" + k] = v
    out["tasks"], out["cnt0"] = sym.tasks(8)
    return out


def test_batch_analysis_equals_the_block_diagonal_analysis():
    """The batched analysis (members analysed alone on several threads, then
    joined) gives exactly what the analysis of the block-diagonal matrix gives
    whole, on every export, for any thread count (empty members included)."""
    probs = inputs.make_batch(count=9, side_lo=3, side_hi=19)
    probs.insert(2, inputs.random_spd_pattern(60, 0.08, seed=5))
    probs.insert(4, inputs.tridiag(1))
    mats = [(p.n, p.colptr, p.rowind, p.perm) for p in probs]
    mats.insert(6, (0, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), None))
    whole = inputs.block_diagonal([dataclasses.replace(p, rhs=None) for p in probs])
    for ratio, cap in ((0.0, 150), (0.2, 7)):
        ref = spchol.analyze(whole.n, whole.colptr, whole.rowind, whole.perm, sn_cap=cap,
                             amalg_ratio=ratio, sched=2)
        want = _whole_analysis_fields(ref)
        for threads in (1, 3, 0):
            bs = spchol.analyze_batch(mats, sn_cap=cap, amalg_ratio=ratio, sched=2,
                                      threads=threads)
            assert bs.info()["nbatch"] == len(mats)
            got = _whole_analysis_fields(bs)
            assert got["info"] == want["info"]
            for k in want:
                if k != "info":
                    assert np.array_equal(got[k], want[k]), (k, ratio, threads)


def test_batch_rejects_bad_member():
    good = inputs.tridiag(5)
    with pytest.raises(spchol.SpcError) as e:
        spchol.analyze_batch([(5, good.colptr, good.rowind, None),
                              (4, [0, 2, 3, 4, 5], [1, 0, 2, 3, 3], None)])
    assert e.value.status == spchol.SPC_ERR_PATTERN
    empty = spchol.analyze_batch([])
    assert empty.info()["n"] == 0 and empty.info()["nbatch"] == 0


@pytest.mark.parametrize("seed", range(6))
def test_batch_analysis_random_mixes(seed):
    """Random mixes of members (random sparse SPD patterns, grids, dense
    blocks, 1x1 and empty matrices) at random options and thread counts: the
    batched analysis equals the block-diagonal matrix's, on every export."""
    rng = np.random.default_rng(900 + seed)
    probs = []
    for k in range(int(rng.integers(3, 14))):
        kind = int(rng.integers(0, 4))
        if kind == 0:
            probs.append(inputs.random_spd_pattern(int(rng.integers(1, 60)),
                                                   float(rng.uniform(0.02, 0.3)),
                                                   seed=int(rng.integers(1 << 30))))
        elif kind == 1:
            probs.extend(inputs.make_batch(count=1, seed=int(rng.integers(1 << 20)), side_lo=2,
                                           side_hi=12))
        elif kind == 2:
            probs.append(inputs.dense_spd(int(rng.integers(1, 30)), seed=int(rng.integers(99))))
        else:
            probs.append(inputs.tridiag(int(rng.integers(1, 40))))
    mats = [(p.n, p.colptr, p.rowind, p.perm) for p in probs]
    if rng.random() < 0.5:
        mats.insert(int(rng.integers(0, len(mats) + 1)),
                    (0, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), None))
    whole = inputs.block_diagonal([dataclasses.replace(p, rhs=None) for p in probs])
    cap = int(rng.choice([1, 5, 16, 150]))
    ratio = float(rng.choice([0.0, 0.1, 0.4]))
    ref = spchol.analyze(whole.n, whole.colptr, whole.rowind, whole.perm, sn_cap=cap,
                         amalg_ratio=ratio, sched=2)
    want = _whole_analysis_fields(ref)
    threads = int(rng.integers(1, 9))
    bs = spchol.analyze_batch(mats, sn_cap=cap, amalg_ratio=ratio, sched=2, threads=threads)
    got = _whole_analysis_fields(bs)
    assert got["info"] == want["info"]
    for k in want:
        if k != "info":
            assert np.array_equal(got[k], want[k]), (k, seed)
    bs.free()
    ref.free()


@pytest.mark.parametrize("y,expect", [(8, [0, 22]), (5, [0, 1, 22]), (11, [0, 1, 2, 22])])
def test_library_amalgamation_refused_then_accepted(y, expect):
    """The library's partition on the hand-worked refusal cases (worked out in
    the oracle pin of the same name): ratio 0.1 merges y = 8 after a refusal
    in the first pass, refuses y = 5 on the parent's accumulated zeros; ratio
    0 leaves the three supernodes alone."""
    p = refusal_case(y)
    ratio = 0.0 if y == 11 else 0.1
    sym = spchol.analyze(p.n, p.colptr, p.rowind, None, sn_cap=150, amalg_ratio=ratio)
    assert sym.export()[2].tolist() == expect


def _paper_dag(sym):
    """Task graph in the paper's notation (Section III-A) from the library's
    exported update pairs: F_s -> U_st -> A_t -> F_t for every pair (s, t)."""
    pr = sym.pairs()
    edges = set()
    for s, t in zip(pr["src"].tolist(), pr["tgt"].tolist()):
        edges |= {(("F", s), ("U", s, t)), (("U", s, t), ("A", t)), (("A", t), ("F", t))}
    return edges


@pytest.mark.parametrize("workers", [1, 2, 256])
def test_fig2_task_graph(workers):
    """Fig. 2 of the paper: supernodes j < i < h where j updates i and h and
    i updates h.  Its edges are F_jj -> U_ji -> A_ii -> F_ii -> U_ih, and
    U_jh, U_ih -> A_hh (-> F_hh), with F_jj -> U_jh.  A dense 3 x 3 matrix with
    a one-column cap gives exactly that: j = 0, i = 1, h = 2.  The device task
    list must hold F, T (panel) and U (tile, with its scatter: U and A fused)
    tasks in an order that respects those edges, with F_hh's counter waiting
    for two update tiles and F_ii's for one."""
    p = inputs.dense_spd(3, seed=1, nrhs=0)
    sym = spchol.analyze(p.n, p.colptr, p.rowind, None, sn_cap=1, sched=2)
    j, i, h = 0, 1, 2
    fig2 = {(("F", j), ("U", j, i)), (("U", j, i), ("A", i)), (("A", i), ("F", i)),
            (("F", i), ("U", i, h)), (("U", j, h), ("A", h)), (("U", i, h), ("A", h)),
            (("F", j), ("U", j, h)), (("A", h), ("F", h))}
    assert _paper_dag(sym) == fig2
    tk, cnt0 = sym.tasks(workers)
    assert cnt0.tolist() == [0, 1, 2]
    order = [tuple(t) for t in tk.tolist()]
    # F(s) = (0, s, 0, 0); T(s, 0) = (1, s, 0, 0); U(s, 0, 0) = (2, s, 0, 0)
    assert order == [(0, j, 0, 0), (1, j, 0, 0), (2, j, 0, 0), (0, i, 0, 0), (1, i, 0, 0),
                     (2, i, 0, 0), (0, h, 0, 0)]


def test_solve_tail_levels():
    """The solves' persistent launch covers the top levels of the supernodal
    elimination tree: only when asked for (solve_tail=1) and in the atomic
    order; every level it covers holds at most 128 supernodes and no small
    one, and the level below it does not (or there is none)."""
    p = inputs.make_grid_problem("lap", (16, 16, 16), 3, sigma=1.0, shift=1e-6, nrhs=1)
    kw = dict(sn_cap=16, amalg_ratio=0.0, small_w=-1)
    assert spchol.analyze(p.n, p.colptr, p.rowind, p.perm, **kw).info()["tail_levels"] == 0
    assert spchol.analyze(p.n, p.colptr, p.rowind, p.perm, solve_tail=1,
                          **kw).info()["tail_levels"] == 0  # deterministic order
    with pytest.raises(spchol.SpcError):
        spchol.analyze(p.n, p.colptr, p.rowind, p.perm, solve_tail=2, **kw)
    for kw2 in (kw, dict(sn_cap=150, amalg_ratio=0.1)):
        sym = spchol.analyze(p.n, p.colptr, p.rowind, p.perm, solve_tail=1, deterministic=0,
                             **kw2)
        info = sym.info()
        _, _, sp, spar = sym.export()
        rp, _ = sym.rows()
        w, r = np.diff(sp), np.diff(rp) - np.diff(sp)
        small = (w <= (16 if kw2.get("small_w", 0) == 0 else 0)) & (r <= 64)
        lev = np.zeros(len(spar), dtype=np.int64)
        for s in range(len(spar)):
            if spar[s] >= 0:
                lev[spar[s]] = max(lev[spar[s]], lev[s] + 1)
        nl = int(lev.max()) + 1
        assert info["nlevels"] == nl
        l0 = nl - info["tail_levels"]
        ok = [np.sum(lev == l) <= 128 and not small[lev == l].any() for l in range(nl)]
        if info["tail_levels"]:
            assert all(ok[l0:]) and (l0 == 0 or not ok[l0 - 1])
            assert info["tail_supernodes"] == int(np.sum(lev >= l0))
        else:
            assert nl - (np.argmin(ok[::-1]) if not all(ok) else nl) < 2
