"""Pins of the oracle's route recovery (smallest minimising predecessor and
backtracked cut points) against enumeration, closed forms and the paper's
worked feasibility example.  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2602_05179_amd import workloads as W

NO = oracle.NO_PRED


def _coords(rng, N):
    xy = rng.integers(0, 1000, size=(N + 1, 2))
    xy[0] = (500, 500)
    return xy


def _matrix(kind, rng, N):
    xy = _coords(rng, N)
    if kind == "round":
        return W.dist_round(xy)
    if kind == "ceil":
        return W.dist_ceil(xy)
    if kind == "l1grid":  # a 4x4 grid under L1: many equal route costs (ties)
        g = rng.integers(0, 4, size=(N + 1, 2))
        g[0] = (2, 2)
        return np.abs(g[:, None, :] - g[None, :, :]).sum(-1).astype(np.int32)
    if kind == "zero":  # every split of equal route count ties
        return np.zeros((N + 1, N + 1), np.int32)
    if kind == "asym":
        d = rng.integers(1, 50, size=(N + 1, N + 1)).astype(np.int32)
        np.fill_diagonal(d, 0)
        return d
    raise ValueError(kind)


def _qvis(dem, tour, s):
    return [int(dem[s, c - 1]) for c in tour]


@pytest.mark.parametrize("kind", ["round", "ceil", "l1grid", "zero", "asym"])
@pytest.mark.parametrize("seed", range(4))
def test_pred_is_smallest_minimiser_by_enumeration(kind, seed):
    """pred(i) = smallest p of the last route over all cheapest splits of
    every prefix (enumeration of all cut sets, n <= 10)."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 11))
    N = n
    dist = _matrix(kind, rng, N)
    tour = (rng.permutation(N) + 1).astype(np.int32)
    Q = int(rng.integers(8, 30))
    dem = rng.integers(0, 12, size=(6, N)).astype(np.int16)
    r = oracle.split_routes(tour, dist, dem, Q)
    for s in range(dem.shape[0]):
        q = _qvis(dem, tour, s)
        want = brute.smallest_last_cut(list(tour), q, dist.tolist(), Q)
        got = [None if int(p) == NO else int(p) for p in r["pred"][s]]
        assert got == want, (kind, seed, s)
        best, _ = brute.best_split(list(tour), q, dist.tolist(), Q)
        k = int(r["nroutes"][s])
        ends = [int(x) for x in r["cuts"][s][:k]]
        assert all(int(x) == 0 for x in r["cuts"][s][k:])
        if best is None:
            assert k == 0 and int(r["costs"][s]) == oracle.INF32
        else:
            assert int(r["costs"][s]) == best
            assert brute.split_cost(list(tour), q, dist.tolist(), Q, ends) == best
            # the cut points follow pred back from n
            chain, i = [], n
            while i > 0:
                chain.append(i)
                i = want[i - 1]
            assert ends == chain[::-1]


def test_paper_feasibility_example_scenario1_routes():
    """Tour (1,2,4,3,5), demands in visiting order (14,15,8,1,8), Q = 17:
    customers 1 and 2 travel alone and 4,3,5 share a route at load exactly
    17.  On a matrix obeying the triangle inequality joining routes never
    costs more, and every other feasible split starts its last route later,
    so the routes end at positions 1, 2, 5 (ties included)."""
    rng = np.random.default_rng(7)
    tour = np.array([1, 2, 4, 3, 5], np.int32)
    qv = [14, 15, 8, 1, 8]
    dem = np.zeros((1, 5), np.int16)
    for pos, c in enumerate(tour):
        dem[0, c - 1] = qv[pos]
    for kind in ("ceil", "l1grid", "zero"):
        dist = _matrix(kind, rng, 5)
        r = oracle.split_routes(tour, dist, dem, 17)
        assert int(r["nroutes"][0]) == 3
        assert [int(x) for x in r["cuts"][0][:3]] == [1, 2, 5]
        assert int(r["pred"][0][4]) == 2 and int(r["pred"][0][1]) == 1 and int(r["pred"][0][0]) == 0


def test_one_route_when_capacity_is_large_on_metric():
    """Q >= total demand on a metric matrix: the single route is cheapest for
    every prefix, so pred(i) = 0 for all i and the only cut is n."""
    rng = np.random.default_rng(11)
    n = 40
    dist = W.dist_ceil(_coords(rng, n))
    tour = (rng.permutation(n) + 1).astype(np.int32)
    dem = rng.integers(1, 10, size=(5, n)).astype(np.int16)
    r = oracle.split_routes(tour, dist, dem, int(dem.sum(axis=1).max()))
    assert (r["pred"] == 0).all()
    assert (r["nroutes"] == 1).all() and (r["cuts"][:, 0] == n).all() and (r["cuts"][:, 1:] == 0).all()


def test_every_pair_over_capacity_gives_one_route_per_customer():
    rng = np.random.default_rng(12)
    n = 30
    dist = W.dist_round(_coords(rng, n))
    tour = (rng.permutation(n) + 1).astype(np.int32)
    dem = rng.integers(6, 11, size=(4, n)).astype(np.int16)  # any two exceed Q = 11
    r = oracle.split_routes(tour, dist, dem, 11)
    assert (r["pred"] == np.arange(n, dtype=np.uint16)[None, :]).all()
    assert (r["nroutes"] == n).all()
    assert (r["cuts"] == np.arange(1, n + 1, dtype=np.uint16)[None, :]).all()


def test_infeasible_scenario_has_no_routes():
    rng = np.random.default_rng(13)
    n = 12
    dist = W.dist_round(_coords(rng, n))
    tour = (rng.permutation(n) + 1).astype(np.int32)
    dem = rng.integers(1, 5, size=(3, n)).astype(np.int16)
    dem[1, tour[4] - 1] = 50  # position 5 alone exceeds Q
    r = oracle.split_routes(tour, dist, dem, 20)
    assert int(r["nroutes"][1]) == 0 and (r["cuts"][1] == 0).all()
    assert int(r["costs"][1]) == oracle.INF32
    assert (r["pred"][1][4:] == NO).all() and (r["pred"][1][:4] != NO).all()
    assert int(r["nroutes"][0]) > 0 and int(r["nroutes"][2]) > 0


def test_routes_costs_match_the_evaluation_oracle():
    """The recovery's costs equal the plain evaluation's on a medium case."""
    inst = W.plain_normal(21, 150, 3000, 120)
    tours, lens, dist, dem = W.as_arrays(inst)
    r = oracle.split_routes(tours, dist, dem, inst.Q, nthreads=4)
    e = oracle.split_eval(tours, lens, dist, dem, inst.Q, nthreads=4)
    assert (r["costs"] == e["costs"][0]).all()
    assert ((r["nroutes"] > 0) == (e["costs"][0] != oracle.INF32)).all()
