"""The batched-factorization autotuner's host logic, with a stand-in timer
(no GPU): size classes, the staged search, the choice of the fastest option
set and the JSON cache."""
import json

import pytest

from paper_1608_00044_amd import inputs, tune


def _mats(count=5, lo=6, hi=14):
    return [(p.n, p.colptr, p.rowind, p.perm)
            for p in inputs.make_batch(count=count, side_lo=lo, side_hi=hi)]


def _fake_timer(cost, calls):
    def timer(mats, values, rhs, precision, opts, steps=2):
        calls.append((precision, dict(opts)))
        return {"ms": cost(opts), "nsup": 1, "levels": 1, "flops_stored": 0.0}
    return timer


def test_size_class_separates_precision_count_size_and_density():
    a = _mats()
    assert tune.size_class(a, 0) == tune.size_class(list(a), 0)
    assert tune.size_class(a, 0) != tune.size_class(a, 1)
    assert tune.size_class(a, 0) != tune.size_class(a * 4, 0)
    assert tune.size_class(a, 0) != tune.size_class(_mats(lo=40, hi=60), 0)
    t = inputs.tridiag(30)
    assert tune.size_class([(t.n, t.colptr, t.rowind, None)] * 5, 0) != tune.size_class(a, 0)
    assert tune.size_class([], 0) == "p0-count0-n0-deg0"


STAGES = (
    (dict(amalg_ratio=0.0), dict(amalg_ratio=0.2)),
    (dict(sn_cap=150), dict(sn_cap=64)),
)
BASE = dict(amalg_ratio=0.0, sn_cap=150)


def _cost(o):
    return {(0.0, 150): 3.0, (0.2, 150): 1.5, (0.2, 64): 2.0, (0.0, 64): 0.5}[
        (o["amalg_ratio"], o["sn_cap"])]


def test_staged_search_and_cache(tmp_path):
    mats = _mats()
    calls = []
    path = str(tmp_path / "sub" / "tune.json")
    best, table = tune.tune_batch(mats, None, None, 1, STAGES, path,
                                  timer=_fake_timer(_cost, calls), base=BASE)
    # stage 0 picks ratio 0.2; stage 1 starts there (the global optimum
    # (0.0, 64) is never visited: the search is coordinate-wise)
    assert best == {"amalg_ratio": 0.2, "sn_cap": 150}
    assert [t["ms"] for t in table] == [3.0, 1.5, 2.0]
    assert [t["stage"] for t in table] == [0, 0, 1]
    # (0.2, 150) is the incumbent of stage 1: timed once only
    assert [c[1] for c in calls] == [dict(amalg_ratio=0.0, sn_cap=150),
                                     dict(amalg_ratio=0.2, sn_cap=150),
                                     dict(amalg_ratio=0.2, sn_cap=64)]
    assert all(c[0] == 1 for c in calls)
    data = json.load(open(path))
    assert list(data) == [tune.size_class(mats, 1)] and data[tune.size_class(mats, 1)]["ms"] == 1.5
    # a second batch of the same class reuses the choice without timing
    calls.clear()
    again, table2 = tune.tune_batch(mats, None, None, 1, STAGES, path,
                                    timer=_fake_timer(_cost, calls), base=BASE)
    assert again == best and table2 is None and calls == []
    # another precision is another class: timed and added beside the first
    tune.tune_batch(mats, None, None, 0, STAGES, path, timer=_fake_timer(_cost, calls),
                    base=BASE)
    assert len(calls) == 3 and len(json.load(open(path))) == 2


def test_default_stages_are_valid_options():
    calls = []
    best, table = tune.tune_batch(_mats(), None, None, 0,
                                  timer=_fake_timer(lambda o: 1.0 + o["amalg_ratio"], calls))
    assert best == tune.BASE
    assert len(table) == len(calls) == len({tuple(sorted(c[1].items())) for c in calls})
    for _, o in calls:
        assert set(o) == set(tune.BASE)
        assert 0.0 <= o["amalg_ratio"] <= 1.0 and 1 <= o["sn_cap"] <= 150
        assert o["small_w"] == -1 or 1 <= o["small_w"] <= 16
        assert 1 <= o["small_r"] <= 64


def test_failing_candidates_are_skipped():
    import math

    import pytest

    from paper_1608_00044_amd.spchol import SPC_ERR_NOT_CONVERGED, SpcError

    def timer(mats, values, rhs, precision, opts, steps=2):
        if opts["amalg_ratio"] == 0.2:
            raise SpcError(SPC_ERR_NOT_CONVERGED, "spc_solve_refine")
        return {"ms": 2.0 + opts["amalg_ratio"], "nsup": 1, "levels": 1, "flops_stored": 0.0}

    best, table = tune.tune_batch(_mats(), None, None, 1, STAGES, timer=timer, base=BASE)
    assert best == {"amalg_ratio": 0.0, "sn_cap": 150}
    bad = [t for t in table if t["options"]["amalg_ratio"] == 0.2]
    assert bad and all(math.isinf(t["ms"]) and t["error"] == SPC_ERR_NOT_CONVERGED for t in bad)

    def always(mats, values, rhs, precision, opts, steps=2):
        raise SpcError(SPC_ERR_NOT_CONVERGED, "spc_solve_refine")

    with pytest.raises(RuntimeError):
        tune.tune_batch(_mats(), None, None, 1, STAGES, timer=always, base=BASE)


def test_default_stages_are_valid_analysis_options():
    """Every candidate of the library's stages (ratio, cap, lane-group split,
    update tile K chunk) is an option set the batched analysis accepts."""
    from paper_1608_00044_amd import inputs, spchol

    chunks = {c["upd_chunk"] for st in tune.STAGES for c in st if "upd_chunk" in c}
    assert chunks == {8, 16, 32}
    probs = inputs.make_batch(count=3, side_lo=16, side_hi=20)
    mats = [(q.n, q.colptr, q.rowind, q.perm) for q in probs]
    for stage in tune.STAGES:
        for cand in stage:
            sym = spchol.analyze_batch(mats, **dict(tune.BASE, **cand))
            assert sym.info()["nbatch"] == 3
            sym.free()
    with pytest.raises(spchol.SpcError):
        spchol.analyze_batch(mats, **dict(tune.BASE, upd_chunk=12))
