"""Seeded synthetic inputs for the scenario-batched split evaluator.

This module only draws inputs: coordinates, integer travel costs, giant
tours and demand scenarios.  It holds none of the split recursion's
arithmetic, so both the CPU oracle (tests) and the HIP path consume the
same arrays without sharing any of the method's code.

Instance shape follows the paper's CVRPSD setting (Sec. 2.3 and App. A):
a depot (node 0) plus customers 1..N, a giant tour that is an ordering of
customers, a scenario-indexed demand for every customer, and a vehicle
capacity Q.  The paper's own instances (CVRPLIB X-set files) are not
available, so these generators stand in for them: integer coordinates on a
[0,1000]^2 grid with a central depot and rounded Euclidean costs.

Layouts (all little-endian, row-major):
  dist     int32 [(N+1), (N+1)]   dist[a, b] = cost of arc a -> b
  tours    int32 [sum(lens)]      concatenated giant tours, ids in 1..N
  lens     int32 [num_tours]
  demands  int16 [S, N]           demands[s, c-1] = demand of customer c
"""
from __future__ import annotations

import dataclasses

import numpy as np

DEPOT_XY = (500, 500)
GRID = 1000


# ----------------------------------------------------------------------------
# coordinates and costs
# ----------------------------------------------------------------------------
def coords(rng: np.random.Generator, N: int, depot=DEPOT_XY, grid=GRID) -> np.ndarray:
    """Integer coordinates, row 0 is the depot, rows 1..N uniform on [0,grid]^2."""
    xy = rng.integers(0, grid + 1, size=(N + 1, 2), dtype=np.int64)
    xy[0] = depot
    return xy


def _sqdist(xy: np.ndarray) -> np.ndarray:
    d = xy[:, None, :] - xy[None, :, :]
    return (d * d).sum(-1)


def _isqrt(m: np.ndarray) -> np.ndarray:
    """Exact integer square root of a non-negative int64 array."""
    r = np.floor(np.sqrt(m.astype(np.float64))).astype(np.int64)
    # correct the float estimate by at most a couple of steps either way
    for _ in range(2):
        r = np.where(r * r > m, r - 1, r)
        r = np.where((r + 1) * (r + 1) <= m, r + 1, r)
    return r


def dist_round(xy: np.ndarray) -> np.ndarray:
    """Nearest-integer Euclidean costs, computed exactly in integers.

    With integer coordinates the squared length m is an integer and never
    equals (k + 1/2)^2, so rounding has no ties: round(sqrt(m)) = r + 1
    exactly when m - r^2 > r, with r = isqrt(m).
    """
    m = _sqdist(xy)
    r = _isqrt(m)
    return (r + (m - r * r > r)).astype(np.int32)


def dist_ceil(xy: np.ndarray) -> np.ndarray:
    """Ceiling Euclidean costs: a metric (ceil(x+y) <= ceil(x)+ceil(y))."""
    m = _sqdist(xy)
    r = _isqrt(m)
    return (r + (r * r < m)).astype(np.int32)


def dist_l1(xy: np.ndarray) -> np.ndarray:
    """Manhattan costs: an integer metric."""
    return np.abs(xy[:, None, :] - xy[None, :, :]).sum(-1).astype(np.int32)


# ----------------------------------------------------------------------------
# tours
# ----------------------------------------------------------------------------
def random_tour(rng: np.random.Generator, N: int, customers=None) -> np.ndarray:
    c = np.arange(1, N + 1) if customers is None else np.asarray(customers)
    return rng.permutation(c).astype(np.int32)


def two_opt_perturb(rng: np.random.Generator, tour: np.ndarray, moves: int) -> np.ndarray:
    """Apply `moves` random segment reversals (2-opt moves) to a copy of tour."""
    t = np.array(tour, dtype=np.int32, copy=True)
    n = t.size
    for _ in range(moves):
        if n < 2:
            break
        i, k = sorted(rng.choice(n, size=2, replace=False))
        t[i:k + 1] = t[i:k + 1][::-1]
    return t


# ----------------------------------------------------------------------------
# demands
# ----------------------------------------------------------------------------
_CHUNK = 1 << 16  # scenarios drawn per chunk (bounds host memory at large S)


def demands_uniform(rng, S: int, N: int, lo: int, hi: int) -> np.ndarray:
    """iid integer demands uniform on [lo, hi]."""
    return rng.integers(lo, hi + 1, size=(S, N), dtype=np.int16)


def demands_normal(rng, S: int, mu: np.ndarray, rel: float = 0.3, lo: int = 1) -> np.ndarray:
    """round(Normal(mu_i, rel*mu_i)) clipped below at `lo`, drawn in chunks."""
    mu = np.asarray(mu, dtype=np.float64)
    out = np.empty((S, mu.size), dtype=np.int16)
    for s0 in range(0, S, _CHUNK):
        s1 = min(S, s0 + _CHUNK)
        x = rng.normal(mu, rel * mu, size=(s1 - s0, mu.size))
        np.rint(x, out=x)
        np.clip(x, lo, 32767, out=x)
        out[s0:s1] = x
    return out


def demands_poisson(rng, S: int, mu: np.ndarray, lo: int = 1) -> np.ndarray:
    """Poisson(mu_i) clipped below at `lo`, drawn in chunks."""
    mu = np.asarray(mu, dtype=np.float64)
    out = np.empty((S, mu.size), dtype=np.int16)
    for s0 in range(0, S, _CHUNK):
        s1 = min(S, s0 + _CHUNK)
        x = rng.poisson(mu, size=(s1 - s0, mu.size))
        np.clip(x, lo, 32767, out=x)
        out[s0:s1] = x
    return out


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Instance:
    """One evaluation call: tours over a shared customer set and scenario set."""
    name: str
    tours: np.ndarray      # int32 [sum(lens)]
    lens: np.ndarray       # int32 [num_tours]
    dist: np.ndarray       # int32 [N+1, N+1]
    demands: np.ndarray    # int16 [S, N]
    Q: int
    seed: int

    @property
    def N(self) -> int:
        return int(self.dist.shape[0] - 1)

    @property
    def S(self) -> int:
        return int(self.demands.shape[0])

    @property
    def num_tours(self) -> int:
        return int(self.lens.size)

    def tour(self, t: int) -> np.ndarray:
        off = int(self.lens[:t].sum())
        return self.tours[off:off + int(self.lens[t])]


def plain_small(seed: int = 1, S: int = 1000) -> Instance:
    """1 tour, n=20, iid demands U{1..10}, Q=30."""
    rng = np.random.default_rng(seed)
    N = 20
    dist = dist_round(coords(rng, N))
    tour = random_tour(rng, N)
    dem = demands_uniform(rng, S, N, 1, 10)
    return Instance("plain n=20 S=%d Q=30" % S, tour, np.array([N], np.int32), dist, dem, 30, seed)


def plain_normal(seed: int, n: int, S: int, Q: int, mu_hi: int = 20) -> Instance:
    """1 tour over n customers, mu_i ~ U{1..mu_hi}, demands round(N(mu,0.3mu)) >= 1."""
    rng = np.random.default_rng(seed)
    dist = dist_round(coords(rng, n))
    tour = random_tour(rng, n)
    mu = rng.integers(1, mu_hi + 1, size=n)
    dem = demands_normal(rng, S, mu)
    return Instance("plain n=%d S=%d Q=%d" % (n, S, Q), tour, np.array([n], np.int32), dist, dem, Q, seed)


def plain_medium(seed: int = 2, S: int = 100_000) -> Instance:
    return plain_normal(seed, 100, S, 100)


def plain_paper_scale(seed: int = 3, S: int = 1_000_000) -> Instance:
    """The paper-scale evaluation: n=200, S=10^6, Q=150."""
    return plain_normal(seed, 200, S, 150)


def batched_ragged(seed: int = 4, num_tours: int = 256, S: int = 10_000,
                   n_lo: int = 50, n_hi: int = 400, Q: int = 100, max_moves: int = 20) -> Instance:
    """Many candidate giant tours of uneven length over one customer pool.

    Pool N = n_hi, one coordinate set, mu_i ~ U[2,15], q = max(1, Poisson(mu_i)).
    Tour t uses customers {1..n_t}, n_t ~ U{n_lo..n_hi}; even t is a random
    permutation, odd t the seed permutation filtered to {1..n_t}; then
    U{0..max_moves} random 2-opt reversals.
    """
    rng = np.random.default_rng(seed)
    N = n_hi
    dist = dist_round(coords(rng, N))
    mu = rng.uniform(2.0, 15.0, size=N)
    dem = demands_poisson(rng, S, mu)
    seed_tour = random_tour(rng, N)
    tours, lens = [], []
    for t in range(num_tours):
        n_t = int(rng.integers(n_lo, n_hi + 1))
        if t % 2 == 0:
            base = random_tour(rng, n_t)
        else:
            base = seed_tour[seed_tour <= n_t]
        tours.append(two_opt_perturb(rng, base, int(rng.integers(0, max_moves + 1))))
        lens.append(n_t)
    return Instance("batched %d tours n=[%d,%d] S=%d Q=%d" % (num_tours, n_lo, n_hi, S, Q),
                    np.concatenate(tours).astype(np.int32), np.array(lens, np.int32),
                    dist, dem, Q, seed)


@dataclasses.dataclass
class Request:
    """One served evaluation request with its own instance."""
    rid: int
    arrival_s: float
    inst: Instance


def served_stream(seed: int = 5, num_requests: int = 10_000, rate_per_s: float = 1000.0,
                  n_lo: int = 50, n_hi: int = 1000, logS_lo: float = 3.0, logS_hi: float = 5.0,
                  Qs=(80, 150, 300)):
    """Poisson-arrival stream of evaluation requests (a generator: instances
    are drawn lazily so a long stream never sits in host memory at once).

    Each request: n ~ U{n_lo..n_hi}, S = round(10^U(logS_lo, logS_hi)),
    Q uniform over Qs, mu_i ~ U{1..20}, demands round(N(mu,0.3mu)) >= 1.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    for rid in range(num_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        n = int(rng.integers(n_lo, n_hi + 1))
        S = int(round(10.0 ** rng.uniform(logS_lo, logS_hi)))
        Q = int(Qs[int(rng.integers(0, len(Qs)))])
        sub = int(rng.integers(0, 2**31 - 1))
        inst = plain_normal(sub, n, S, Q)
        inst.name = "served rid=%d n=%d S=%d Q=%d" % (rid, n, S, Q)
        yield Request(rid, t, inst)


def as_arrays(inst: Instance):
    """Contiguous arrays in the C-ABI layout."""
    return (np.ascontiguousarray(inst.tours, np.int32), np.ascontiguousarray(inst.lens, np.int32),
            np.ascontiguousarray(inst.dist, np.int32), np.ascontiguousarray(inst.demands, np.int16))


@dataclasses.dataclass
class InventoryInstance:
    """Order-up-to inventory reinsertion instance: B = customers x scenarios
    independent problems over T days with inventory states 0..U."""
    name: str
    U: int
    demand: np.ndarray    # int32 [T, B]
    opt_cost: np.ndarray  # int32 [T, B, R] insertion cost of each route option
    opt_cap: np.ndarray   # int32 [T, B, R] residual capacity of each route option
    h: np.ndarray         # int32 [U+1] end-of-day cost of each inventory level
    u: int                # unit transport cost
    rho: int              # unit shortage penalty
    I0: np.ndarray        # int32 [B] initial inventories
    seed: int


def inventory_ou(seed: int = 6, customers: int = 100, scenarios: int = 1000, U: int = 20, T: int = 7,
                 R: int = 4) -> InventoryInstance:
    """Per customer: daily demand mean mu ~ U[1, U/3], demands Poisson(mu)
    clipped to [0, U + 2] per day and scenario; holding cost h ~ U{1..5} per
    unit, shortage penalty 4 h per unit (rho > 1 times holding); R route
    options per day and scenario with insertion costs U{5..60} and residual
    capacities U{0..U}; unit transport cost 1; initial inventory U{0..U}.
    Problem b = c * scenarios + s."""
    rng = np.random.default_rng(seed)
    B = customers * scenarios
    mu = rng.uniform(1.0, max(1.0, U / 3.0), size=customers)
    lam = np.repeat(mu, scenarios)
    demand = np.minimum(rng.poisson(lam[None, :], size=(T, B)), U + 2).astype(np.int32)
    hc = rng.integers(1, 6, size=customers)
    # one h table per instance: the mean customer's holding cost (tables are shared)
    h = (int(np.round(hc.mean())) * np.arange(U + 1)).astype(np.int32)
    rho = 4 * int(np.round(hc.mean()))
    opt_cost = rng.integers(5, 61, size=(T, B, R)).astype(np.int32)
    opt_cap = rng.integers(0, U + 1, size=(T, B, R)).astype(np.int32)
    I0 = np.repeat(rng.integers(0, U + 1, size=customers), scenarios).astype(np.int32)
    return InventoryInstance("inventory OU %d customers x %d scenarios U=%d T=%d R=%d" % (customers, scenarios, U, T, R),
                             U, demand, opt_cost, opt_cap, h, 1, rho, I0, seed)
