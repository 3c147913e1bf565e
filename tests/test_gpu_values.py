"""GPU parity of the full value table (split_values_device, through the C
ABI) against the CPU oracle's split_values, scenario by scenario.

Bit-exact: every V_s(j), j = 1..n, SPLIT_INF where the oracle reports +inf.
The GPU writes V position-major ([n, S]).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2602_05179_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_05179_amd import binding as b
    return b


def _gpu_values(binding, tour, dist, dem, Q):
    t, d, q = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (tour, dist, dem))
    V, status = binding.split_values_device(t, d, q, Q)
    torch.cuda.synchronize()
    return V.cpu().numpy(), int(status.cpu().item())


def _oracle_table(tour, dist, dem, Q, inf):
    n, S = tour.size, dem.shape[0]
    ref = np.empty((n, S), np.int64)
    for s in range(S):
        vals, _ = oracle.split_values(tour, dist, dem[s, tour - 1], Q)
        ref[:, s] = [inf if v is None else v for v in vals[1:]]
    return ref


def _check(binding, tour, dist, dem, Q, label):
    _say("%s n=%d N=%d S=%d Q=%d" % (label, tour.size, dist.shape[0] - 1, dem.shape[0], Q))
    got, status = _gpu_values(binding, tour, dist, dem, Q)
    ref = _oracle_table(tour, dist, dem, Q, binding.SPLIT_INF)
    assert status == 0, label
    bad = np.argwhere(got != ref)
    assert bad.size == 0, "%s: %d mismatches, first (j-1, s)=%s got %d want %d" % (
        label, len(bad), bad[0], got[tuple(bad[0])], ref[tuple(bad[0])])
    return got


def test_values_several_tiles_and_ragged_tail(binding):
    inst = W.plain_normal(31, 40, 300, 60)  # 5 tiles, the last with 44 scenarios
    tours, lens, dist, dem = W.as_arrays(inst)
    _check(binding, tours, dist, dem, inst.Q, "plain n=40")


def test_values_infeasible_scenarios_and_wide_demands(binding):
    rng = np.random.default_rng(32)
    N, S, Q = 30, 130, 50
    dist = W.dist_round(W.coords(rng, N))
    dem = rng.integers(0, 40, size=(S, N)).astype(np.int16)
    dem[5, 7] = 51          # one customer above Q: +inf from its position on
    dem[70, :3] = 300       # values above a byte
    tour = W.random_tour(rng, N)
    _check(binding, tour, dist, dem, Q, "infeasible and wide")


def test_values_long_windows(binding):
    """Windows far longer than a register ring (zero demands admit every
    predecessor)."""
    rng = np.random.default_rng(33)
    N, S = 90, 70
    dist = W.dist_round(W.coords(rng, N))
    dem = rng.integers(0, 2, size=(S, N)).astype(np.int16)
    tour = W.random_tour(rng, N)
    _check(binding, tour, dist, dem, 1000, "long windows")


def test_values_last_row_equals_evaluator(binding):
    inst = W.plain_normal(34, 200, 2000, 150)
    tours, lens, dist, dem = W.as_arrays(inst)
    got, status = _gpu_values(binding, tours, dist, dem, inst.Q)
    assert status == 0
    ref = oracle.split_eval(tours, lens, dist, dem, inst.Q)
    assert np.array_equal(got[-1], ref["costs"][0])


def test_values_invalid_tour_and_negative_demand(binding):
    rng = np.random.default_rng(35)
    N, S, Q = 12, 80, 30
    dist = W.dist_round(W.coords(rng, N))
    dem = rng.integers(1, 8, size=(S, N)).astype(np.int16)
    tour = W.random_tour(rng, N)
    bad = tour.copy()
    bad[4] = N + 3
    got, status = _gpu_values(binding, bad, dist, dem, Q)
    assert (got == binding.SPLIT_INF).all()
    dem2 = dem.copy()
    dem2[9, tour[2] - 1] = -1
    got, status = _gpu_values(binding, tour, dist, dem2, Q)
    assert status == 1
    assert (got[:, 9] == binding.SPLIT_INF).all()
    keep = np.arange(S) != 9
    ref = _oracle_table(tour, dist, dem[keep], Q, binding.SPLIT_INF)
    assert np.array_equal(got[:, keep], ref)


def test_values_empty_tour(binding):
    rng = np.random.default_rng(36)
    dist = W.dist_round(W.coords(rng, 5))
    dem = rng.integers(1, 5, size=(10, 5)).astype(np.int16)
    got, status = _gpu_values(binding, np.zeros(0, np.int32), dist, dem, 10)
    assert got.shape == (0, 10) and status == 0
