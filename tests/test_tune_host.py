"""The batched-factorization autotuner's host logic, with a stand-in timer
(no GPU): size classes, the choice of the fastest candidate and the JSON
cache."""
import json

from paper_1608_00044_amd import inputs, tune


def _mats(count=5, lo=6, hi=14):
    return [(p.n, p.colptr, p.rowind, p.perm)
            for p in inputs.make_batch(count=count, side_lo=lo, side_hi=hi)]


def _fake_timer(costs, calls):
    def timer(mats, values, rhs, precision, opts, steps=2):
        calls.append((precision, opts["amalg_ratio"], opts["sn_cap"]))
        return {"ms": costs[(opts["amalg_ratio"], opts["sn_cap"])], "nsup": 1, "levels": 1,
                "flops_stored": 0.0}
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


def test_tuner_picks_the_fastest_and_caches_it(tmp_path):
    mats = _mats()
    cands = (dict(amalg_ratio=0.0, sn_cap=150), dict(amalg_ratio=0.2, sn_cap=150),
             dict(amalg_ratio=0.2, sn_cap=64))
    costs = {(0.0, 150): 3.0, (0.2, 150): 1.5, (0.2, 64): 2.0}
    calls = []
    path = str(tmp_path / "sub" / "tune.json")
    best, table = tune.tune_batch(mats, None, None, 1, cands, path, timer=_fake_timer(costs, calls))
    assert best == {"amalg_ratio": 0.2, "sn_cap": 150}
    assert [t["ms"] for t in table] == [3.0, 1.5, 2.0]
    assert calls == [(1, 0.0, 150), (1, 0.2, 150), (1, 0.2, 64)]
    data = json.load(open(path))
    assert list(data) == [tune.size_class(mats, 1)]
    # a second batch of the same class reuses the choice without timing
    calls.clear()
    again, table2 = tune.tune_batch(mats, None, None, 1, cands, path,
                                    timer=_fake_timer(costs, calls))
    assert again == best and table2 is None and calls == []
    # another precision is another class: timed and added beside the first
    tune.tune_batch(mats, None, None, 0, cands, path, timer=_fake_timer(costs, calls))
    assert len(calls) == 3 and len(json.load(open(path))) == 2


def test_tuner_without_cache_always_times():
    calls = []
    costs = {(r, c): 1.0 + r for r, c in [(o["amalg_ratio"], o["sn_cap"])
                                           for o in tune.CANDIDATES]}
    best, table = tune.tune_batch(_mats(), None, None, 0, timer=_fake_timer(costs, calls))
    assert best == {"amalg_ratio": 0.0, "sn_cap": 150}
    assert len(table) == len(tune.CANDIDATES) == len(calls)
    for o in tune.CANDIDATES:
        assert 0.0 <= o["amalg_ratio"] <= 1.0 and 1 <= o["sn_cap"] <= 150
