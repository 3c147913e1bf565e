"""The first-stage candidate search (genetic algorithm over giant tours) on
the CPU, with the oracle as its evaluator: determinism, elitism, candidate
counts, permutation validity, and the reported best sum against a fresh
oracle evaluation."""
import numpy as np
import pytest

import oracle
from paper_2602_05179_amd import binding
from paper_2602_05179_amd import workloads as W


def _oracle_eval(dist, dem, Q):
    def ev(tours):
        count, n = tours.shape
        lens = np.full(count, n, np.int32)
        return oracle.split_eval(tours.ravel(), lens, dist, dem, Q, nthreads=4)["sums"]
    return ev


def _run(inst, **kw):
    tours, lens, dist, dem = W.as_arrays(inst)
    return binding.search(dist, dem, inst.Q, evaluator=_oracle_eval(dist, dem, inst.Q), **kw)


def test_search_is_deterministic_elitist_and_consistent():
    inst = W.plain_normal(41, 25, 300, 40)
    kw = dict(population=12, offspring=20, generations=15, mutation=0.4, seed=7)
    a = _run(inst, **kw)
    b = _run(inst, **kw)
    assert np.array_equal(a["best_tour"], b["best_tour"]) and a["best_sum"] == b["best_sum"]
    assert np.array_equal(a["trace"][:, 1:], b["trace"][:, 1:])
    assert sorted(a["best_tour"].tolist()) == list(range(1, 26))
    assert a["candidates"] == 12 + 15 * 20
    tr = a["trace"]
    assert tr.shape == (16, 3) and (np.diff(tr[:, 2]) <= 0).all() and (np.diff(tr[:, 1]) == 20).all()
    assert tr[-1, 2] == a["best_sum"] < tr[0, 2]
    tours, lens, dist, dem = W.as_arrays(inst)
    again = oracle.split_eval(a["best_tour"], np.array([25], np.int32), dist, dem, inst.Q)["sums"][0]
    assert again == a["best_sum"]


def test_search_seeds_and_initial_tour():
    inst = W.plain_normal(42, 20, 200, 35)
    a = _run(inst, population=8, offspring=8, generations=5, seed=1)
    b = _run(inst, population=8, offspring=8, generations=5, seed=2)
    assert not np.array_equal(a["trace"][:, 2], b["trace"][:, 2]) or not np.array_equal(a["best_tour"], b["best_tour"])
    # an initial tour seeds the population: the result is never worse than it
    init = inst.tours[:20].copy()
    tours, lens, dist, dem = W.as_arrays(inst)
    init_sum = oracle.split_eval(init, np.array([20], np.int32), dist, dem, inst.Q)["sums"][0]
    c = _run(inst, population=8, offspring=8, generations=3, seed=3, init_tour=init)
    assert c["best_sum"] <= init_sum


def test_search_rejects_bad_parameters():
    inst = W.plain_normal(43, 10, 50, 30)
    with pytest.raises(binding.SplitError):
        _run(inst, population=1, offspring=4, generations=2)
    with pytest.raises(binding.SplitError):
        _run(inst, population=4, offspring=4, generations=0, time_budget_s=0)
    with pytest.raises(binding.SplitError):
        _run(inst, population=4, offspring=4, generations=2, init_tour=np.arange(10, dtype=np.int32))  # has 0
    with pytest.raises(binding.SplitError):
        _run(inst, population=4, offspring=4, generations=2, mutation=1.5)


def test_search_time_budget_stops():
    inst = W.plain_normal(44, 15, 100, 30)
    r = _run(inst, population=6, offspring=6, generations=0, time_budget_s=0.3, seed=5)
    assert r["trace"][-1, 0] < 5.0 and r["candidates"] == 6 + 6 * (len(r["trace"]) - 1)
