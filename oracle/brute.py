"""Brute-force split values by enumerating every set of cut points.

TEST INFRASTRUCTURE ONLY (pins the C oracle; never used by the product).

Independent of the dynamic programme: a split of the prefix sigma_1..sigma_j
is a set of cut positions among 1..j-1; each maximal segment is one route
depot -> sigma_a .. sigma_b -> depot (paper Sec. 2.3, route cost W) and is
admissible only if its load is at most Q.  The value of the prefix is the
cheapest admissible split, computed here by trying all 2^(j-1) cut sets.
"""
from __future__ import annotations

INF = None  # no admissible split


def route_cost(seg, dist):
    """depot -> seg[0] -> ... -> seg[-1] -> depot."""
    c = dist[0][seg[0]] + dist[seg[-1]][0]
    for a, b in zip(seg[:-1], seg[1:]):
        c += dist[a][b]
    return c


def best_split(tour, qvis, dist, Q):
    """(cost, routes) of the cheapest admissible split of the whole tour, or
    (None, None).  qvis[k] is the demand of tour[k]."""
    n = len(tour)
    if n == 0:
        return 0, []
    best, arg = None, None
    for mask in range(1 << (n - 1)):
        cuts = [k + 1 for k in range(n - 1) if mask >> k & 1]
        bounds = [0] + cuts + [n]
        total, routes, ok = 0, [], True
        for a, b in zip(bounds[:-1], bounds[1:]):
            if sum(qvis[a:b]) > Q:
                ok = False
                break
            total += route_cost(tour[a:b], dist)
            routes.append(tuple(tour[a:b]))
        if ok and (best is None or total < best):
            best, arg = total, routes
    return best, arg


def prefix_values(tour, qvis, dist, Q):
    """[V(0), V(1), ..., V(n)] with None where no admissible split exists."""
    return [best_split(tour[:j], qvis[:j], dist, Q)[0] for j in range(len(tour) + 1)]


def feasible_pairs(qvis, Q):
    """Number of (p, j) with p < j and sum(q[p..j-1]) <= Q, by direct count."""
    n = len(qvis)
    return sum(1 for j in range(1, n + 1) for p in range(j) if sum(qvis[p:j]) <= Q)


def all_splits(n):
    """Every cut set of n customers as a tuple of (a, b) half-open segments."""
    for mask in range(1 << max(n - 1, 0)):
        cuts = [k + 1 for k in range(n - 1) if mask >> k & 1]
        bounds = [0] + cuts + [n]
        yield tuple(zip(bounds[:-1], bounds[1:]))


def smallest_last_cut(tour, qvis, dist, Q):
    """For every prefix j = 1..n: the smallest p such that some cheapest
    admissible split of sigma_1..sigma_j has its last route p+1..j (None if
    the prefix has no admissible split).  By enumeration of all cut sets of
    each prefix, independent of any recursion."""
    out = []
    for j in range(1, len(tour) + 1):
        best, starts = None, set()
        for mask in range(1 << (j - 1)):
            cuts = [k + 1 for k in range(j - 1) if mask >> k & 1]
            bounds = [0] + cuts + [j]
            total, ok = 0, True
            for a, b in zip(bounds[:-1], bounds[1:]):
                if sum(qvis[a:b]) > Q:
                    ok = False
                    break
                total += route_cost(tour[a:b], dist)
            if not ok:
                continue
            if best is None or total < best:
                best, starts = total, {bounds[-2]}
            elif total == best:
                starts.add(bounds[-2])
        out.append(min(starts) if best is not None else None)
    return out


def split_cost(tour, qvis, dist, Q, ends):
    """Cost of the split whose routes end at positions `ends` (increasing,
    last = n), or None if a route is over capacity or `ends` is malformed."""
    n = len(tour)
    if not ends or ends[-1] != n or any(b <= a for a, b in zip([0] + ends[:-1], ends)):
        return None
    total = 0
    for a, b in zip([0] + ends[:-1], ends):
        if sum(qvis[a:b]) > Q:
            return None
        total += route_cost(tour[a:b], dist)
    return total


def best_split_variant(tour, qvis, dist, Q, beta=-1, K=0):
    """Cheapest split over ALL cut sets with at most K routes (K = 0: any
    number), each route paying beta * max(0, load - Q) (beta < 0: routes over
    Q excluded).  None if no cut set qualifies.  Enumeration, independent of
    any recursion."""
    n = len(tour)
    if n == 0:
        return 0
    best = None
    for mask in range(1 << (n - 1)):
        cuts = [k + 1 for k in range(n - 1) if mask >> k & 1]
        if K and len(cuts) + 1 > K:
            continue
        bounds = [0] + cuts + [n]
        total, ok = 0, True
        for a, b in zip(bounds[:-1], bounds[1:]):
            load = sum(qvis[a:b])
            if load > Q:
                if beta < 0:
                    ok = False
                    break
                total += beta * (load - Q)
            total += route_cost(tour[a:b], dist)
        if ok and (best is None or total < best):
            best = total
    return best
