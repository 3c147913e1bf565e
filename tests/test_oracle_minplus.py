"""Pins of the min-plus oracle and the order-up-to inventory instance: the
paper's two worked examples, enumeration of state paths and of delivery
decisions, tie and saturation rules.  CPU only."""
import numpy as np
import pytest

from oracle import minplus as M

INF = M.INF


def test_paper_illustrative_update():
    """App. A illustrative example: J = (0, 1, 3), A with one infeasible
    entry; the update gives (2, 3), with a tie in the first column."""
    J = np.array([[0, 1, 3]])
    A = np.array([[2, 5], [1, INF], [3, 0]])
    out, arg = M.minplus_step(A, J)
    assert out.tolist() == [[2, 3]]
    assert arg.tolist() == [[0, 2]]  # 2 + 0 and 1 + 1 tie: the smaller source wins


def test_paper_inventory_example():
    """App. B illustrative matrix form: U = 2, initial inventory 1, demand 1
    per day, transport q, end-of-day costs (5, 1, 0); two days give (5, 2,
    +inf) then (7, 4, +inf), terminal cost 4, delivering on both days."""
    A_paper = np.array([[5, 3, INF], [5, 2, INF], [INF, 1, INF]])
    T, B = 2, 1
    demand = np.ones((T, B), np.int64)
    cost = np.zeros((T, B, 1), np.int64)
    cap = np.full((T, B, 1), 2, np.int64)
    A = M.ou_transitions(2, demand, cost, cap, h=[5, 1, 0], u=1, rho=0)
    assert (A[0, 0] == A_paper).all() and (A[1, 0] == A_paper).all()
    J1 = np.array([[INF, 0, INF]])
    J2, _ = M.minplus_step(A[0], J1)
    assert J2.tolist() == [[5, 2, INF]]
    J3, args = M.minplus_forward(A, J1, shared=False)
    assert J3.tolist() == [[7, 4, INF]]
    assert J3.min() == 4
    path = M.backtrack(J3, args)
    assert path[:, 0].tolist() == [1, 1, 1]  # replenish to full each day, end at 1
    assert M.ou_brute(2, [1], demand, cost, cap, [5, 1, 0], 1, 0).tolist() == [4]


@pytest.mark.parametrize("shared", [True, False])
@pytest.mark.parametrize("seed", range(6))
def test_forward_equals_path_enumeration(shared, seed):
    rng = np.random.default_rng(seed)
    T, m, B = int(rng.integers(1, 5)), int(rng.integers(1, 5)), 3
    shape = (T, m, m) if shared else (T, B, m, m)
    A = rng.integers(0, 6, size=shape).astype(np.int64)
    A[rng.random(shape) < 0.35] = INF
    J0 = rng.integers(0, 4, size=(B, m)).astype(np.int64)
    J0[rng.random((B, m)) < 0.3] = INF
    JT, args = M.minplus_forward(A, J0, shared)
    assert (JT == M.brute_paths(A, J0, shared)).all()
    # the backtracked path realises J_T at its final state
    path = M.backtrack(JT, args)
    for b in range(B):
        if JT[b].min() >= INF:
            assert (path[:, b] == -1).all()
            continue
        c = J0[b, path[0, b]]
        for t in range(T):
            c += A[t, path[t, b], path[t + 1, b]] if shared else A[t, b, path[t, b], path[t + 1, b]]
        assert c == JT[b].min()


def test_ties_and_saturation():
    A = np.array([[3, INF], [1, INF], [INF, INF]])
    J = np.array([[1, 3, 0]])
    out, arg = M.minplus_step(A, J)
    assert out.tolist() == [[4, INF]] and arg.tolist() == [[0, -1]]
    big = np.array([[INF - 5]])
    out, arg = M.minplus_step(big, np.array([[10]]))
    assert out.tolist() == [[INF]] and arg.tolist() == [[-1]]  # finite sum past INF is +inf
    out, _ = M.minplus_step(np.array([[INF - 11]]), np.array([[10]]))
    assert out.tolist() == [[INF - 1]]


@pytest.mark.parametrize("seed", range(8))
def test_inventory_forward_equals_decision_enumeration(seed):
    rng = np.random.default_rng(100 + seed)
    T, B, R = int(rng.integers(1, 6)), 4, int(rng.integers(1, 4))
    U = int(rng.integers(1, 7))
    demand = rng.integers(0, U + 2, size=(T, B))
    cost = rng.integers(0, 20, size=(T, B, R))
    cap = rng.integers(0, U + 1, size=(T, B, R))
    h = rng.integers(0, 8, size=U + 1)
    u, rho = int(rng.integers(0, 3)), int(rng.integers(0, 10))
    I0 = rng.integers(0, U + 1, size=B)
    A = M.ou_transitions(U, demand, cost, cap, h, u, rho)
    J0 = np.full((B, U + 1), INF, np.int64)
    J0[np.arange(B), I0] = 0
    JT, _ = M.minplus_forward(A, J0, shared=False)
    assert (JT.min(axis=1) == M.ou_brute(U, I0, demand, cost, cap, h, u, rho)).all()


def _golden_ou(golden_dir):
    import json
    import os
    g = json.load(open(os.path.join(golden_dir, "ou_two_options_stockout.json")))
    fix = lambda rows: np.array([[INF if v is None else v for v in r] for r in rows], np.int64)
    return g, fix


def test_two_option_stockout_golden(golden_dir):
    """Three route options and stock-outs (App. B: A(I,J) = min_r A(I,J;r),
    penalty per unit of unmet demand).  U = 3, h = (0, 2, 3, 9), u = 1,
    rho = 5; options (cost, residual capacity) = (10, 2), (4, 1), (7, 3).

    transport(q) = cheapest option that carries q, plus q:
      q = 1: every option carries it, cheapest 4 -> 5;
      q = 2: options 1 and 3 carry it, cheapest 7 -> 9;
      q = 3: only option 3 carries it -> 10.
    Day 1, demand 2 (row I, no delivery | deliver up to 3):
      I = 0: stay -> J = 0, unmet 2: 0 + h0 + 10 = 10 | q = 3 -> J = 1: 10 + h1 = 12
      I = 1: stay -> J = 0, unmet 1: 5               | q = 2 -> J = 1: 9 + h1 = 11
      I = 2: stay -> J = 0: h0 = 0                   | q = 1 -> J = 1: 5 + h1 = 7
      I = 3: stay -> J = 1: h1 = 2                   | (nothing to deliver)
    Day 2, demand 5 (every choice ends at J = 0):
      I = 0: stay, unmet 5: 25 | q = 3, unmet 2: 10 + 10 = 20  -> 20
      I = 1: stay, unmet 4: 20 | q = 2, unmet 2: 9 + 10 = 19   -> 19
      I = 2: stay, unmet 3: 15 | q = 1, unmet 2: 5 + 10 = 15   -> 15
      I = 3: stay, unmet 2: 10                                 -> 10
    From I0 = 0: after day 1 (10, 12, inf, inf); after day 2
    J(0) = min(10 + 20, 12 + 19) = 30 (skip day 1, deliver on day 2).

    A first-option-with-room rule (10 for q = 2), a strict capacity test
    (no option for q = 3, option 3 for q = 1), or a dropped or mis-signed
    stock-out term each changes one of these entries."""
    g, fix = _golden_ou(golden_dir)
    T, B, R = 2, 1, 3
    demand = np.array(g["demand"], np.int64).reshape(T, B)
    cost = np.broadcast_to(np.array(g["options"]["cost"], np.int64), (T, B, R)).copy()
    cap = np.broadcast_to(np.array(g["options"]["cap"], np.int64), (T, B, R)).copy()
    A = M.ou_transitions(g["U"], demand, cost, cap, g["h"], g["u"], g["rho"])
    assert (A[0, 0] == fix(g["A_day1"])).all()
    assert (A[1, 0] == fix(g["A_day2"])).all()
    J0 = np.full((B, g["U"] + 1), INF, np.int64)
    J0[0, g["I0"]] = 0
    J1, _ = M.minplus_step(A[0], J0)
    assert (J1 == fix([g["J_after_day1"]])).all()
    J2, _ = M.minplus_forward(A, J0, shared=False)
    assert (J2 == fix([g["J_after_day2"]])).all()
    assert int(J2.min()) == g["best_total"]
    assert M.ou_brute(g["U"], [g["I0"]], demand, cost, cap, g["h"], g["u"], g["rho"]).tolist() == [30]


@pytest.mark.parametrize("seed", range(6))
def test_several_options_equal_elementwise_min_of_single_options(seed):
    """App. B note (ii): the transition matrix over R route options equals
    the elementwise minimum of the R matrices built with one option each
    (each of the single-option form the paper's inventory example pins)."""
    rng = np.random.default_rng(300 + seed)
    T, B, R = 3, 4, int(rng.integers(2, 5))
    U = int(rng.integers(1, 8))
    demand = rng.integers(0, U + 3, size=(T, B))
    cost = rng.integers(0, 30, size=(T, B, R))
    cap = rng.integers(0, U + 1, size=(T, B, R))
    h = rng.integers(0, 9, size=U + 1)
    u, rho = int(rng.integers(0, 3)), int(rng.integers(0, 7))
    A = M.ou_transitions(U, demand, cost, cap, h, u, rho)
    singles = [M.ou_transitions(U, demand, cost[:, :, r:r + 1], cap[:, :, r:r + 1], h, u, rho)
               for r in range(R)]
    assert (A == np.minimum.reduce(singles)).all()
