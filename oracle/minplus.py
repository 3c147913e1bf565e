"""Min-plus Bellman updates and the order-up-to inventory instance: plain
numpy definitions.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU leg use this module; it shares nothing with the HIP library.

Values are int64 here; INF (= 2^31 - 1, the library's +inf) marks an
infeasible entry, and any finite sum that reaches INF is reported as INF
(the library's int32 saturation rule).

Forward update (Sec. 2, "Min-Plus Matrix Formulation"; App. A,
"Illustrative example for the min-plus matrix-vector Bellman update"):
    J_{t+1}(j) = min_i  A_t(i, j) + J_t(i),
with +inf when every term is +inf.  arg_t(j) is the smallest i attaining it
(-1 when J_{t+1}(j) is +inf).  A path is recovered from the smallest
minimising final state backwards through arg.

Order-up-to inventory instance (App. B: each day a customer is either
replenished up to its capacity U or not at all; the illustrative matrix
form of its DP): states are end-of-day inventories 0..U.  From inventory I
with day demand d, the delivery q is 0 or U - I; the next state is
max(0, I + q - d); the day costs
    transport(q) + h[next] + rho * max(0, d - I - q),
with transport(0) = 0 and transport(q) = min over the day's route options r
whose residual capacity is at least q of c_r, plus u * q (no such route:
delivery impossible).  A_t(I, J) is the cheapest such choice landing in J.
"""
import itertools

import numpy as np

INF = (1 << 31) - 1


def _sat(x):
    x = np.asarray(x, dtype=np.int64)
    return np.where(x >= INF, INF, x)


def minplus_step(A, J):
    """One update for a batch: A [B, m, m'] (or [m, m'] shared), J [B, m] ->
    (J' [B, m'], arg [B, m'])."""
    A = np.asarray(A, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    if A.ndim == 2:
        A = np.broadcast_to(A, (J.shape[0],) + A.shape)
    terms = np.where((A >= INF) | (J[:, :, None] >= INF), INF, _sat(A + J[:, :, None]))
    out = terms.min(axis=1)
    arg = terms.argmin(axis=1)  # first (smallest) i among equal minima
    arg = np.where(out >= INF, -1, arg)
    return out, arg


def minplus_forward(A, J0, shared):
    """A: [T, m, m] if shared else [T, B, m, m]; J0 [B, m].  Returns (J_T,
    args [T, B, m])."""
    J = np.asarray(J0, dtype=np.int64)
    args = []
    for t in range(A.shape[0]):
        J, arg = minplus_step(A[t], J)
        args.append(arg)
    return J, np.array(args, dtype=np.int64).reshape(len(args), J.shape[0], -1)


def backtrack(JT, args):
    """State path [T+1, B]: the smallest minimising final state, then back
    through the recorded minimisers; -1 throughout when J_T is all +inf."""
    T, B = args.shape[0], JT.shape[0]
    path = np.full((T + 1, B), -1, np.int64)
    for b in range(B):
        if JT[b].min() >= INF:
            continue
        s = int(np.argmin(JT[b]))
        path[T, b] = s
        for t in range(T - 1, -1, -1):
            s = int(args[t, b, s])
            path[t, b] = s
    return path


def brute_paths(A, J0, shared):
    """Cheapest cost of reaching each final state over all m^T state paths."""
    A = np.asarray(A, dtype=np.int64)
    J0 = np.asarray(J0, dtype=np.int64)
    T = A.shape[0]
    B, m = J0.shape
    out = np.full((B, m), INF, np.int64)
    for b in range(B):
        for path in itertools.product(range(m), repeat=T + 1):
            c = int(J0[b, path[0]])
            if c >= INF:
                continue
            ok = True
            for t in range(T):
                a = int(A[t, path[t], path[t + 1]] if shared else A[t, b, path[t], path[t + 1]])
                if a >= INF:
                    ok = False
                    break
                c += a
            if ok and c < INF:
                out[b, path[-1]] = min(out[b, path[-1]], c)
    return out


def ou_transport(q, costs, caps, u):
    """transport(q) for one day: min c_r over options with cap_r >= q, plus u*q."""
    if q == 0:
        return 0
    best = INF
    for c, cap in zip(costs, caps):
        if cap >= q and c < best:
            best = int(c)
    return INF if best >= INF else best + u * q


def ou_transitions(U, demand, opt_cost, opt_cap, h, u, rho):
    """A [T, B, U+1, U+1] of the order-up-to instance.
    demand [T, B]; opt_cost, opt_cap [T, B, R]; h [U+1]."""
    demand = np.asarray(demand)
    T, B = demand.shape
    m = U + 1
    A = np.full((T, B, m, m), INF, np.int64)
    for t in range(T):
        for b in range(B):
            d = int(demand[t, b])
            for I in range(m):
                for q in sorted({0, U - I}):
                    tr = ou_transport(q, opt_cost[t, b], opt_cap[t, b], u)
                    if tr >= INF:
                        continue
                    J = max(0, I + q - d)
                    c = tr + int(h[J]) + rho * max(0, d - I - q)
                    if c < A[t, b, I, J]:
                        A[t, b, I, J] = min(c, INF)
    return A


def ou_brute(U, I0, demand, opt_cost, opt_cap, h, u, rho):
    """Cheapest total over all delivery decisions for every batch element, by
    enumeration: each day either no delivery or a delivery up to U on one
    chosen route option r (admissible when its residual capacity holds the
    delivery).  The route option is part of the enumerated decision, so the
    minimum over options is reached by enumeration instead of through
    `ou_transport`, and the unmet demand is written as demand minus what the
    stock on hand serves."""
    demand = np.asarray(demand)
    T, B = demand.shape
    R = np.asarray(opt_cost).shape[2]
    out = np.full(B, INF, np.int64)
    for b in range(B):
        # a decision per day: -1 = no delivery, r >= 0 = deliver on option r
        for dec in itertools.product(range(-1, R), repeat=T):
            stock, total, ok = int(I0[b]), 0, True
            for t in range(T):
                d = int(demand[t, b])
                r = dec[t]
                if r < 0:
                    q = 0
                else:
                    q = U - stock
                    if q == 0 or int(opt_cap[t, b, r]) < q:
                        ok = False  # a delivery of nothing, or one the route cannot carry
                        break
                    total += int(opt_cost[t, b, r]) + u * q
                on_hand = stock + q
                served = min(on_hand, d)
                stock = on_hand - served
                total += int(h[stock]) + rho * (d - served)
            if ok:
                out[b] = min(out[b], total)
    return np.where(out >= INF, INF, out)
