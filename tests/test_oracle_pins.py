"""Pins for the CPU oracle against what the paper and mathematics fix.

None of these tests touches the GPU.  Every check compares the oracle with
something other than itself: the paper's worked examples (golden fixtures),
an independent brute-force enumeration of all cut sets, closed forms that
hold on metric cost matrices, and invariants of the recursion.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2602_05179_amd import workloads as W

INF32 = oracle.INF32


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def _qvis(tour, demand_row):
    return [int(demand_row[c - 1]) for c in tour]


def _W(tour, dist, p, j):
    """Route cost of tour positions p+1..j (1-based), from the paper's formula."""
    return brute.route_cost(list(tour[p:j]), dist)


# ----------------------------------------------------------------------------
# the paper's worked split example (App. A)
# ----------------------------------------------------------------------------
def test_w2_masked_transition_entries(golden_dir):
    g = _load(golden_dir, "w2_split_toy.json")
    tour, q, Q, dist = g["tour"], g["demands_visiting_order"], g["Q"], g["dist"]
    for key, want in g["A"].items():
        p, i = map(int, key.split(","))
        load = sum(q[p:i])
        got = brute.route_cost(tour[p:i], dist) if load <= Q else None
        assert got == want, key


def test_w2_values_match_paper(golden_dir):
    g = _load(golden_dir, "w2_split_toy.json")
    V, cells = oracle.split_values(g["tour"], np.array(g["dist"]), g["demands_visiting_order"], g["Q"])
    assert V == g["V"]
    # feasible (p,i): (0,1),(0,2),(1,2),(2,3)
    assert cells == 4
    assert brute.prefix_values(g["tour"], g["demands_visiting_order"], g["dist"], g["Q"]) == g["V"]


def test_w2_load_equal_to_capacity_is_feasible(golden_dir):
    g = _load(golden_dir, "w2_split_toy.json")
    # with Q=4 the route (sigma_1, sigma_2) of load 5 is no longer admissible
    V4, _ = oracle.split_values(g["tour"], np.array(g["dist"]), g["demands_visiting_order"], 4)
    assert V4[2] == 2 + 4  # two single routes
    V5, _ = oracle.split_values(g["tour"], np.array(g["dist"]), g["demands_visiting_order"], 5)
    assert V5[2] == 4


def test_w3_scenario1_closed_form_on_metric(golden_dir):
    g = _load(golden_dir, "w3_feasibility.json")
    tour, Q = g["tour"], g["Q"]
    q = g["scenario_1"]["demands_visiting_order"]
    routes = g["scenario_1"]["routes"]
    rng = np.random.default_rng(7)
    for k in range(20):
        xy = W.coords(rng, 5)
        dist = (W.dist_ceil if k % 2 else W.dist_l1)(xy)
        V, _ = oracle.split_values(tour, dist, q, Q)
        want = sum(brute.route_cost(list(r), dist) for r in routes)
        assert V[5] == want


def test_w3_scenario_m_printed_split_is_feasible(golden_dir):
    g = _load(golden_dir, "w3_feasibility.json")
    tour, Q = g["tour"], g["Q"]
    q = g["scenario_m"]["demands_visiting_order"]
    routes = g["scenario_m"]["routes"]
    # each printed route respects Q
    pos = 0
    for r in routes:
        assert sum(q[pos:pos + len(r)]) <= Q
        pos += len(r)
    rng = np.random.default_rng(8)
    for _ in range(10):
        dist = W.dist_round(W.coords(rng, 5))
        V, _ = oracle.split_values(tour, dist, q, Q)
        assert V[5] <= sum(brute.route_cost(list(r), dist) for r in routes)


# ----------------------------------------------------------------------------
# brute force over every cut set
# ----------------------------------------------------------------------------
def _random_matrix(rng, N, kind):
    if kind == "round":
        return W.dist_round(W.coords(rng, N))
    if kind == "ceil":
        return W.dist_ceil(W.coords(rng, N))
    if kind == "asym":
        d = rng.integers(0, 50, size=(N + 1, N + 1)).astype(np.int32)
        np.fill_diagonal(d, 0)
        return d
    if kind == "zero":
        return np.zeros((N + 1, N + 1), np.int32)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["round", "ceil", "asym", "zero"])
def test_prefix_values_equal_brute_force(kind):
    rng = np.random.default_rng(11)
    for trial in range(60):
        n = int(rng.integers(1, 10))
        N = n + int(rng.integers(0, 3))
        dist = _random_matrix(rng, N, kind)
        tour = rng.choice(np.arange(1, N + 1), size=n, replace=False).astype(np.int32)
        qvis = rng.integers(0, 9, size=n).tolist()
        Q = int(rng.integers(0, 25))
        V, cells = oracle.split_values(tour, dist, qvis, Q)
        Vb = brute.prefix_values(tour.tolist(), qvis, dist.tolist(), Q)
        assert V == Vb, (trial, tour, qvis, Q)
        assert cells == brute.feasible_pairs(qvis, Q)
        Vn, cells_nb = oracle.split_values(tour, dist, qvis, Q, use_break=False)
        assert Vn == V and cells_nb == cells


def test_brute_force_n12_full_tour():
    rng = np.random.default_rng(12)
    for _ in range(3):
        N = 12
        dist = W.dist_round(W.coords(rng, N))
        tour = W.random_tour(rng, N)
        qvis = rng.integers(1, 11, size=N).tolist()
        V, _ = oracle.split_values(tour, dist, qvis, 30)
        assert V[-1] == brute.best_split(tour.tolist(), qvis, dist.tolist(), 30)[0]


def test_scenario_api_matches_brute_force():
    """split_eval gathers demands by customer id and reduces exactly."""
    rng = np.random.default_rng(13)
    N, S = 8, 50
    dist = W.dist_round(W.coords(rng, N))
    tours = [W.random_tour(rng, N), W.random_tour(rng, N)[:5]]
    lens = np.array([t.size for t in tours], np.int32)
    dem = W.demands_uniform(rng, S, N, 1, 9)
    Q = 15
    r = oracle.split_eval(np.concatenate(tours), lens, dist, dem, Q)
    for t, tour in enumerate(tours):
        want = [brute.best_split(tour.tolist(), _qvis(tour, dem[s]), dist.tolist(), Q)[0] for s in range(S)]
        assert r["costs"][t].tolist() == want
        assert r["sums"][t] == sum(want)
        assert r["means"][t] == sum(want) / S


# ----------------------------------------------------------------------------
# closed forms and special cases
# ----------------------------------------------------------------------------
def test_infinite_capacity_gives_single_route_on_metric():
    rng = np.random.default_rng(21)
    for _ in range(30):
        N = int(rng.integers(1, 40))
        dist = W.dist_ceil(W.coords(rng, N))
        tour = W.random_tour(rng, N)
        qvis = rng.integers(1, 20, size=N)
        V, _ = oracle.split_values(tour, dist, qvis, int(qvis.sum()))
        for j in range(1, N + 1):
            assert V[j] == _W(tour, dist.tolist(), 0, j)


def test_every_pair_over_capacity_gives_out_and_back_routes():
    rng = np.random.default_rng(22)
    for _ in range(30):
        N = int(rng.integers(1, 40))
        dist = W.dist_round(W.coords(rng, N))
        tour = W.random_tour(rng, N)
        Q = 10
        qvis = rng.integers(6, 11, size=N)  # q <= Q, any two consecutive > Q
        V, _ = oracle.split_values(tour, dist, qvis, Q)
        assert V[N] == sum(int(dist[0, c]) + int(dist[c, 0]) for c in tour)


def test_demand_above_capacity_is_infeasible():
    rng = np.random.default_rng(23)
    N, S = 15, 40
    dist = W.dist_round(W.coords(rng, N))
    tour = W.random_tour(rng, N)
    dem = W.demands_uniform(rng, S, N, 1, 5)
    dem[7, 3] = 31
    r = oracle.split_eval(tour, [N], dist, dem, 30)
    assert r["costs"][0, 7] == INF32
    assert (r["costs"][0, np.arange(S) != 7] < INF32).all()
    assert r["sums"][0] == oracle.INF64
    assert np.isinf(r["means"][0])


def test_empty_tour_costs_zero():
    dist = np.zeros((4, 4), np.int32)
    dem = np.ones((3, 3), np.int16)
    r = oracle.split_eval(np.zeros(0, np.int32), [0], dist, dem, 5)
    assert r["costs"].tolist() == [[0, 0, 0]] and r["sums"][0] == 0 and r["means"][0] == 0.0


def test_zero_demands_and_zero_capacity():
    rng = np.random.default_rng(24)
    N = 9
    dist = W.dist_ceil(W.coords(rng, N))
    tour = W.random_tour(rng, N)
    V, _ = oracle.split_values(tour, dist, [0] * N, 0)
    assert V[N] == _W(tour, dist.tolist(), 0, N)


# ----------------------------------------------------------------------------
# invariants of the recursion
# ----------------------------------------------------------------------------
def test_monotone_in_prefix_on_metric_and_relaxed_on_rounded():
    rng = np.random.default_rng(31)
    for k in range(200):
        N = int(rng.integers(2, 30))
        xy = W.coords(rng, N)
        tour = W.random_tour(rng, N)
        qvis = rng.integers(1, 11, size=N)
        Vm, _ = oracle.split_values(tour, W.dist_ceil(xy), qvis, 30)
        assert all(a <= b for a, b in zip(Vm[:-1], Vm[1:]))
        Vr, _ = oracle.split_values(tour, W.dist_round(xy), qvis, 30)
        # each rounding is off by at most 1/2, so d(a,c) <= d(a,b) + d(b,c) + 1
        assert all(a <= b + 1 for a, b in zip(Vr[:-1], Vr[1:]))
        single = _W(tour, W.dist_round(xy).tolist(), 0, N)
        Vinf, _ = oracle.split_values(tour, W.dist_round(xy), qvis, int(qvis.sum()))
        assert single - (N - 1) <= Vinf[N] <= single


def test_monotone_in_capacity_and_demand():
    rng = np.random.default_rng(32)
    for _ in range(100):
        N = int(rng.integers(1, 25))
        dist = W.dist_round(W.coords(rng, N))
        tour = W.random_tour(rng, N)
        qvis = rng.integers(1, 11, size=N)
        Q = int(rng.integers(10, 40))
        v0 = oracle.split_values(tour, dist, qvis, Q)[0][N]
        v1 = oracle.split_values(tour, dist, qvis, Q + int(rng.integers(1, 10)))[0][N]
        assert v0 is None or v1 <= v0
        q2 = qvis.copy()
        q2[int(rng.integers(0, N))] += int(rng.integers(1, 5))
        v2 = oracle.split_values(tour, dist, q2, Q)[0][N]
        assert v0 is None or v2 is None or v2 >= v0
        if v2 is not None:
            assert v0 is not None


def test_scenario_permutation_and_tour_reversal():
    rng = np.random.default_rng(33)
    N, S = 25, 64
    xy = W.coords(rng, N)
    dist = W.dist_round(xy)  # symmetric
    tour = W.random_tour(rng, N)
    dem = W.demands_uniform(rng, S, N, 1, 10)
    r = oracle.split_eval(tour, [N], dist, dem, 30)
    perm = rng.permutation(S)
    rp = oracle.split_eval(tour, [N], dist, dem[perm], 30)
    assert (rp["costs"][0] == r["costs"][0][perm]).all()
    assert rp["sums"][0] == r["sums"][0] and rp["means"][0] == r["means"][0]
    rr = oracle.split_eval(tour[::-1].copy(), [N], dist, dem, 30)
    assert (rr["costs"] == r["costs"]).all()


def test_threads_do_not_change_results():
    inst = W.plain_medium(2, S=3000)
    a = oracle.split_eval(inst.tours, inst.lens, inst.dist, inst.demands, inst.Q, nthreads=1)
    b = oracle.split_eval(inst.tours, inst.lens, inst.dist, inst.demands, inst.Q, nthreads=5)
    for k in a:
        assert (a[k] == b[k]).all()


def test_invalid_arguments_are_rejected():
    dist = np.zeros((4, 4), np.int32)
    dem = np.ones((2, 3), np.int16)
    with pytest.raises(oracle.OracleError):
        oracle.split_eval(np.array([1, 4], np.int32), [2], dist, dem, 5)
    with pytest.raises(oracle.OracleError):
        oracle.split_eval(np.array([1, 2], np.int32), [2], dist, dem, -1)
