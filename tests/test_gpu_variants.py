"""GPU parity of the split variants (soft capacity with an overload penalty,
a fleet of at most K routes) through the C ABI against the CPU oracle.
Bit-exact per-scenario costs; the status word for invalid inputs."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2602_05179_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
INF32 = np.iinfo(np.int32).max


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_05179_amd import binding as b
    return b


def _gpu(binding, tour, dist, dem, Q, beta, K):
    t, d, q = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (tour, dist, dem))
    out = binding.split_variant_device(t, d, q, Q, beta=beta, K=K)
    torch.cuda.synchronize()
    return out.costs.cpu().numpy(), int(out.status.cpu()[0])


def _ref(tour, dist, dem, Q, beta, K):
    r = oracle.split_variant(tour, dist, dem, Q, beta=beta, K=K, nthreads=THREADS)
    out = np.where(r == oracle.INF64, INF32, r)
    assert (out <= INF32).all()
    return out.astype(np.int32)


def _check(binding, tour, dist, dem, Q, beta, K, label):
    _say("%s n=%d N=%d S=%d Q=%d beta=%d K=%d" % (label, tour.size, dist.shape[0] - 1, dem.shape[0], Q, beta, K))
    got, status = _gpu(binding, tour, dist, dem, Q, beta, K)
    assert status == 0, (label, status)
    ref = _ref(tour, dist, dem, Q, beta, K)
    bad = np.flatnonzero(got != ref)
    assert bad.size == 0, "%s: %d mismatches, first s=%d got %d want %d" % (
        label, bad.size, bad[0], got[bad[0]], ref[bad[0]])
    return got


def _one(inst):
    tours, lens, dist, dem = W.as_arrays(inst)
    return tours[:int(lens[0])], dist, dem


MODES = [(-1, 0), (-1, 1), (-1, 3), (-1, 9), (0, 0), (4, 0), (4, 5), (60, 0), (2, 14)]


@pytest.mark.parametrize("beta,K", MODES)
def test_variant_modes_small(binding, beta, K):
    inst = W.plain_small(1, S=1000)
    _check(binding, *_one(inst), inst.Q, beta, K, "small")


@pytest.mark.parametrize("beta,K", MODES)
@pytest.mark.parametrize("Q", [60, 250])
def test_variant_modes_ragged(binding, beta, K, Q):
    inst = W.plain_normal(70 + Q, 90, 64 * 11 + 13, Q)
    _check(binding, *_one(inst), Q, beta, K, "n=90 ragged")


def test_hard_unlimited_equals_the_evaluator(binding):
    inst = W.plain_normal(71, 150, 5000, 120)
    tour, dist, dem = _one(inst)
    got, status = _gpu(binding, tour, dist, dem, inst.Q, -1, 0)
    assert status == 0
    t, l, d, q = (torch.from_numpy(np.ascontiguousarray(a)).cuda()
                  for a in (tour, np.array([tour.size], np.int32), dist, dem))
    ev = binding.split_eval_device(t, l, d, q, inst.Q)
    torch.cuda.synchronize()
    assert np.array_equal(ev.costs.cpu().numpy()[0], got)


def test_variant_paper_scale_sampled(binding):
    """n=200, S=10^6, Q=150: soft capacity, a fleet bound, and both
    together (the configurations the benchmark times) on the full scenario
    set, checked on 3000 sampled scenarios."""
    inst = W.plain_paper_scale(3, S=1_000_000)
    tour, dist, dem = _one(inst)
    rng = np.random.default_rng(9)
    idx = np.sort(rng.choice(dem.shape[0], size=3000, replace=False))
    idx[-1] = dem.shape[0] - 1  # the ragged last tile
    for beta, K in ((10, 0), (-1, 25), (10, 25)):
        _say("paper scale beta=%d K=%d" % (beta, K))
        got, status = _gpu(binding, tour, dist, dem, inst.Q, beta, K)
        assert status == 0
        ref = _ref(tour, dist, dem[idx], inst.Q, beta, K)
        assert np.array_equal(got[idx], ref)


def test_variant_fleet_of_n_equals_unlimited(binding):
    inst = W.plain_normal(72, 40, 900, 50)
    tour, dist, dem = _one(inst)
    for beta in (-1, 3):
        a, _ = _gpu(binding, tour, dist, dem, inst.Q, beta, 0)
        b, _ = _gpu(binding, tour, dist, dem, inst.Q, beta, 40)
        c, _ = _gpu(binding, tour, dist, dem, inst.Q, beta, 500)
        assert np.array_equal(a, b) and np.array_equal(a, c)


# ----------------------------------------------------------------------------
# the exact fallback
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("beta,K", [(-1, 0), (5, 0), (-1, 4), (5, 3)])
def test_variant_windows_past_the_ring(binding, beta, K):
    inst = W.plain_normal(73, 100, 64 * 4 + 9, 1500)  # hard windows of ~100 positions
    _check(binding, *_one(inst), inst.Q, beta, K, "long windows")


def test_variant_mixed_overflow_and_wide_demands(binding):
    rng = np.random.default_rng(74)
    N = n = 80
    dist = W.dist_round(W.coords(rng, N))
    tour = (rng.permutation(N) + 1).astype(np.int32)
    dem = rng.integers(1, 12, size=(64 * 8, N)).astype(np.int16)
    dem[64 * 2:64 * 3] = 1                                     # one tile with long windows
    dem[64 * 5:64 * 6] = rng.integers(200, 400, size=(64, N))  # one tile past a byte
    for beta, K in ((-1, 0), (7, 0), (-1, 12), (7, 6)):
        Q = 60 if beta < 0 else 45
        if beta < 0:
            d2 = dem.copy()
            d2[64 * 5:64 * 6] = rng.integers(1, 50, size=(64, N))  # keep hard capacity feasible
        else:
            d2 = dem
        _check(binding, tour, dist, d2, Q, beta, K, "mixed")


def test_variant_pool_too_large_for_lds(binding):
    rng = np.random.default_rng(75)
    N, n = 3000, 60
    dist = W.dist_round(W.coords(rng, N))
    tour = (rng.permutation(N)[:n] + 1).astype(np.int32)
    dem = rng.integers(1, 20, size=(130, N)).astype(np.int16)
    for beta, K in ((-1, 0), (3, 4)):
        _check(binding, tour, dist, dem, 70, beta, K, "N=3000")


# ----------------------------------------------------------------------------
# both demand paths forced: the tile in LDS (1) and the tour-ordered copy
# streamed from the workspace (2)
# ----------------------------------------------------------------------------
def _path_mixed():
    rng = np.random.default_rng(80)
    N, n = 110, 83  # a tour over part of the pool
    dist = W.dist_round(W.coords(rng, N))
    tour = (rng.permutation(N)[:n] + 1).astype(np.int32)
    dem = rng.integers(1, 12, size=(64 * 7 + 11, N)).astype(np.int16)
    dem[64 * 2:64 * 3] = 1                       # a tile with long hard windows
    dem[64 * 4 + 3, tour[30] - 1] = 280          # a demand past a byte
    return tour, dist, dem


@pytest.mark.parametrize("beta,K", [(-1, 0), (-1, 4), (-1, 9), (3, 0), (3, 5)])
@pytest.mark.parametrize("Q", [60, 250])
@pytest.mark.parametrize("path", [1, 2])
def test_variant_forced_path(binding, path, Q, beta, K):
    inst = W.plain_normal(81 + Q, 120, 64 * 6 + 21, Q)
    tour, dist, dem = _one(inst)
    binding.set_variant_path(path)
    try:
        _check(binding, tour, dist, dem, Q, beta, K, "path %d" % path)
        if Q == 60:
            tour, dist, dem = _path_mixed()
            _check(binding, tour, dist, dem, 45, beta, K, "path %d mixed" % path)
    finally:
        binding.set_variant_path(0)


@pytest.mark.parametrize("path", [1, 2])
def test_variant_forced_path_long_tour_and_n1(binding, path):
    inst = W.plain_normal(83, 600, 64 * 2 + 5, 150)
    tour, dist, dem = _one(inst)
    rng = np.random.default_rng(84)
    d9 = W.dist_round(W.coords(rng, 9))
    q9 = rng.integers(0, 6, size=(130, 9)).astype(np.int16)
    binding.set_variant_path(path)
    try:
        for beta, K in ((-1, 0), (4, 0), (-1, 30), (4, 7)):
            _check(binding, tour, dist, dem, 150, beta, K, "path %d n=600" % path)
            _check(binding, np.array([4], np.int32), d9, q9, 3, beta, K, "path %d n=1" % path)
    finally:
        binding.set_variant_path(0)


@pytest.mark.parametrize("beta,K", [(-1, 0), (6, 0), (-1, 25), (6, 12)])
def test_variant_ordered_path_many_tiles(binding, beta, K):
    """n = N = 1000 takes the tour-ordered path by itself (120 tiles plus a
    ragged one), every scenario against the oracle."""
    inst = W.plain_normal(86, 1000, 64 * 120 + 9, 150)
    tour, dist, dem = _one(inst)
    _check(binding, tour, dist, dem, inst.Q, beta, K, "ordered path n=1000")


def test_variant_ordered_path_invalid_demand(binding):
    rng = np.random.default_rng(85)
    N = n = 300
    dist = W.dist_round(W.coords(rng, N))
    tour = (rng.permutation(N) + 1).astype(np.int32)
    dem = rng.integers(1, 10, size=(200, N)).astype(np.int16)
    dem[120, tour[5] - 1] = -2
    binding.set_variant_path(2)
    try:
        got, status = _gpu(binding, tour, dist, dem, 30, 4, 3)
        assert status & binding.VARIANT_BAD_DEMAND and (got == INF32).all()
        dem[120, tour[5] - 1] = 2
        _check(binding, tour, dist, dem, 30, 4, 3, "ordered, valid after invalid")
    finally:
        binding.set_variant_path(0)


# ----------------------------------------------------------------------------
# degenerate cases and validation
# ----------------------------------------------------------------------------
def test_variant_empty_and_single(binding):
    dist = np.zeros((4, 4), np.int32)
    dem = np.ones((70, 3), np.int16)
    for beta, K in ((-1, 0), (5, 2)):
        got, status = _gpu(binding, np.zeros(0, np.int32), dist, dem, 5, beta, K)
        assert status == 0 and (got == 0).all()
    rng = np.random.default_rng(76)
    dist = W.dist_round(W.coords(rng, 9))
    dem = rng.integers(0, 6, size=(130, 9)).astype(np.int16)
    for beta, K in ((-1, 0), (2, 0), (-1, 1), (2, 1)):
        _check(binding, np.array([4], np.int32), dist, dem, 3, beta, K, "n=1")


def test_variant_hard_fleet_too_small_is_infinite(binding):
    rng = np.random.default_rng(77)
    N = n = 30
    dist = W.dist_round(W.coords(rng, N))
    tour = (rng.permutation(N) + 1).astype(np.int32)
    dem = rng.integers(5, 10, size=(200, N)).astype(np.int16)
    got = _check(binding, tour, dist, dem, 20, -1, 2, "fleet too small")
    assert (got == INF32).all()  # total load >= 150 needs more than 2 routes of 20


def test_variant_invalid_inputs_set_status(binding):
    rng = np.random.default_rng(78)
    N = n = 30
    dist = W.dist_round(W.coords(rng, N))
    tour = (rng.permutation(N) + 1).astype(np.int32)
    dem = rng.integers(1, 10, size=(200, N)).astype(np.int16)
    bad = tour.copy()
    bad[2] = N + 3
    got, status = _gpu(binding, bad, dist, dem, 30, 4, 0)
    assert status & binding.VARIANT_BAD_TOUR and (got == INF32).all()
    neg = dem.copy()
    neg[120, tour[5] - 1] = -2  # its tile fails the byte staging and takes the exact path
    got, status = _gpu(binding, tour, dist, neg, 30, 4, 0)
    assert status & binding.VARIANT_BAD_DEMAND and (got == INF32).all()
    big = np.full((100, N), 30000, np.int16)  # load 900000 + Q: beta * (load + Q) >= 2^29
    got, status = _gpu(binding, tour, dist, big, 30, 1000, 0)
    assert status & binding.VARIANT_PENALTY_RANGE and (got == INF32).all()
    # a valid call on the same process afterwards
    _check(binding, tour, dist, dem, 30, 4, 0, "valid after invalid")


def test_variant_rejects_bad_scalars(binding):
    rng = np.random.default_rng(79)
    dist = W.dist_round(W.coords(rng, 5))
    dem = np.ones((10, 5), np.int16)
    t, d, q = (torch.from_numpy(a).cuda() for a in (np.arange(1, 6, dtype=np.int32), dist, dem))
    with pytest.raises(binding.SplitError):
        binding.split_variant_device(t, d, q, 5, beta=1 << 24)
    with pytest.raises(binding.SplitError):
        binding.split_variant_device(t, d, q, 5, K=-1)
