"""GPU parity of route recovery (through the C ABI) against the CPU oracle.

Bit-exact: per-scenario costs, every predecessor pred_s(i) (smallest
minimising p, 0xFFFF where V_s(i) is +inf), the number of routes, and the
route ends up to that number.  The GPU writes pred and cuts position-major
([n, S]); the oracle scenario-major ([S, n]).
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2602_05179_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_05179_amd import binding as b
    return b


def _gpu_routes(binding, tour, dist, dem, Q):
    t, d, q = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (tour, dist, dem))
    out = binding.split_routes_device(t, d, q, Q)
    torch.cuda.synchronize()
    return out.host()


def _assert_routes_equal(got, ref, label):
    n = got["pred"].shape[0]
    bad = np.argwhere(got["costs"] != ref["costs"])
    assert bad.size == 0, "%s: %d cost mismatches, first s=%d got %d want %d" % (
        label, len(bad), bad[0][0], got["costs"][bad[0][0]], ref["costs"][bad[0][0]])
    gp = got["pred"].T
    bad = np.argwhere(gp != ref["pred"])
    assert bad.size == 0, "%s: %d pred mismatches, first (s, i-1)=%s got %d want %d" % (
        label, len(bad), bad[0], gp[tuple(bad[0])], ref["pred"][tuple(bad[0])])
    assert np.array_equal(got["nroutes"], ref["nroutes"]), label
    mask = np.arange(n)[:, None] < got["nroutes"][None, :]
    assert np.array_equal(got["cuts"][mask], ref["cuts"].T[mask]), label


def _check(binding, tour, dist, dem, Q, label):
    _say("%s n=%d N=%d S=%d Q=%d" % (label, tour.size, dist.shape[0] - 1, dem.shape[0], Q))
    got = _gpu_routes(binding, tour, dist, dem, Q)
    ref = oracle.split_routes(tour, dist, dem, Q, nthreads=THREADS)
    _assert_routes_equal(got, ref, label)
    return got, ref


def _inst_arrays(inst):
    tours, lens, dist, dem = W.as_arrays(inst)
    return tours[:int(lens[0])], dist, dem


def _coords(rng, N):
    return W.coords(rng, N)


# ----------------------------------------------------------------------------
# named workloads and shapes
# ----------------------------------------------------------------------------
def test_routes_small(binding):
    inst = W.plain_small(1, S=1000)
    _check(binding, *_inst_arrays(inst), inst.Q, "plain n=20 S=1000")


def test_routes_ragged_tail_and_multiple_tiles(binding):
    inst = W.plain_normal(31, 150, 64 * 37 + 29, 120)
    got, _ = _check(binding, *_inst_arrays(inst), inst.Q, "n=150 ragged S")
    assert (got["nroutes"] > 1).all()


def test_routes_paper_scale_full(binding):
    """n=200, S=10^6, Q=150: every scenario against the oracle, and the
    costs equal the evaluator's."""
    inst = W.plain_paper_scale(3, S=1_000_000)
    tour, dist, dem = _inst_arrays(inst)
    got, _ = _check(binding, tour, dist, dem, inst.Q, "paper scale n=200 S=1e6")
    t, l, d, q = (torch.from_numpy(np.ascontiguousarray(a)).cuda()
                  for a in (tour, np.array([tour.size], np.int32), dist, dem))
    ev = binding.split_eval_device(t, l, d, q, inst.Q)
    torch.cuda.synchronize()
    assert np.array_equal(ev.costs.cpu().numpy()[0], got["costs"])


@pytest.mark.parametrize("variant_idx", range(4))
@pytest.mark.parametrize("Q", [100, 300])
def test_every_route_variant(binding, variant_idx, Q):
    vs = binding.ROUTE_VARIANTS
    if variant_idx >= len(vs):
        pytest.skip("fewer variants compiled")
    inst = W.plain_normal(40 + Q, 120, 3000, Q)
    binding.set_route_variant(*vs[variant_idx])
    try:
        _check(binding, *_inst_arrays(inst), Q, "variant %s Q=%d" % (vs[variant_idx], Q))
    finally:
        binding.set_route_variant(0)


# ----------------------------------------------------------------------------
# ties: the smallest-p rule
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["zero", "l1grid", "const"])
def test_routes_ties(binding, kind):
    rng = np.random.default_rng(77)
    n = N = 90
    if kind == "zero":
        dist = np.zeros((N + 1, N + 1), np.int32)
    elif kind == "const":
        dist = np.full((N + 1, N + 1), 5, np.int32)
        np.fill_diagonal(dist, 0)
    else:
        g = rng.integers(0, 3, size=(N + 1, 2))
        dist = np.abs(g[:, None, :] - g[None, :, :]).sum(-1).astype(np.int32)
    tour = (rng.permutation(N) + 1).astype(np.int32)
    dem = rng.integers(0, 9, size=(700, N)).astype(np.int16)
    for Q in (12, 40):
        got, _ = _check(binding, tour, dist, dem, Q, "ties %s Q=%d" % (kind, Q))


# ----------------------------------------------------------------------------
# the exact fallback: windows past the ring, demands past a byte, large pools
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("scale,Q", [(100, 100), (100, 300), (14, 300), (14, 100)])
def test_routes_wide_costs(binding, scale, Q):
    """Costs too wide for packed keys: scale 100 puts 3 n maxcost past 2^23
    (both rings take the per-cell argmin path); scale 14 puts it between 2^22
    and 2^23 (ring 32 packs keys, ring 64 does not)."""
    rng = np.random.default_rng(60 + scale)
    N = n = 100
    dist = W.dist_round(_coords(rng, N) * scale)
    tour = (rng.permutation(N) + 1).astype(np.int32)
    maxc = int(max(dist[0, tour].max(), dist[tour, 0].max(), dist[tour[:-1], tour[1:]].max()))
    assert 3 * n * maxc < 1 << 29
    if scale == 14:
        assert (1 << 22) <= 3 * n * maxc < (1 << 23)
    else:
        assert 3 * n * maxc >= 1 << 23
    dem = rng.integers(1, 15, size=(64 * 9 + 5, N)).astype(np.int16)
    _check(binding, tour, dist, dem, Q, "wide costs x%d Q=%d" % (scale, Q))


def test_routes_window_past_the_ring(binding):
    inst = W.plain_normal(51, 160, 900, 2500)  # windows of ~200 positions
    for v in ((32, 8, 3, 3), (64, 16, 4, 4)):
        binding.set_route_variant(*v)
        try:
            _check(binding, *_inst_arrays(inst), inst.Q, "long windows %s" % (v,))
        finally:
            binding.set_route_variant(0)


def test_routes_mixed_ring_overflow_per_tile(binding):
    """Only some tiles have windows past the ring."""
    rng = np.random.default_rng(52)
    N = n = 100
    dist = W.dist_round(_coords(rng, N))
    tour = (rng.permutation(N) + 1).astype(np.int32)
    dem = rng.integers(1, 12, size=(64 * 12, N)).astype(np.int16)
    dem[64 * 3:64 * 4] = 1   # windows of length Q
    dem[64 * 7 + 5] = 0      # one scenario: every prefix admissible
    _check(binding, tour, dist, dem, 60, "mixed overflow")


def test_routes_demands_past_a_byte(binding):
    rng = np.random.default_rng(53)
    N = n = 70
    dist = W.dist_ceil(_coords(rng, N))
    tour = (rng.permutation(N) + 1).astype(np.int32)
    dem = rng.integers(100, 400, size=(64 * 5 + 3, N)).astype(np.int16)
    dem[:64] = rng.integers(1, 40, size=(64, N))  # first tile fits a byte
    _check(binding, tour, dist, dem, 1000, "demands > 255")


def test_routes_pool_too_large_for_lds(binding):
    rng = np.random.default_rng(54)
    N, n = 3000, 80
    dist = W.dist_round(_coords(rng, N))
    tour = (rng.permutation(N)[:n] + 1).astype(np.int32)
    dem = rng.integers(1, 20, size=(150, N)).astype(np.int16)
    _check(binding, tour, dist, dem, 70, "N=3000 no LDS tile")


def test_routes_long_tour(binding):
    inst = W.plain_normal(55, 1000, 64 * 6 + 1, 150)
    _check(binding, *_inst_arrays(inst), inst.Q, "n=1000")


# ----------------------------------------------------------------------------
# both demand paths forced: the tile in LDS (1) and the tour-ordered copy
# streamed from the workspace (2)
# ----------------------------------------------------------------------------
def _case_ragged():
    inst = W.plain_normal(61, 150, 64 * 13 + 29, 120)
    return _inst_arrays(inst) + (inst.Q,)


def _case_wide(scale, Q):
    rng = np.random.default_rng(62 + scale)
    N = n = 100
    dist = W.dist_round(_coords(rng, N) * scale)
    tour = (rng.permutation(N) + 1).astype(np.int32)
    return tour, dist, rng.integers(1, 15, size=(64 * 5 + 5, N)).astype(np.int16), Q


def _case_mixed():
    rng = np.random.default_rng(63)
    N, n = 130, 97  # a tour over part of the pool
    dist = W.dist_round(_coords(rng, N))
    tour = (rng.permutation(N)[:n] + 1).astype(np.int32)
    dem = rng.integers(1, 12, size=(64 * 8 + 3, N)).astype(np.int16)
    dem[64 * 2:64 * 3] = 1          # windows past ring 32
    dem[64 * 5 + 1, tour[40] - 1] = 300  # a demand past a byte
    dem[64 * 6:64 * 7:5, tour[7] - 1] = 70  # position 8 alone exceeds Q
    return tour, dist, dem, 60


def _case_long():
    inst = W.plain_normal(64, 1000, 64 * 4 + 7, 150)
    return _inst_arrays(inst) + (inst.Q,)


def _case_short():
    rng = np.random.default_rng(65)
    N = 9
    dist = W.dist_round(_coords(rng, N))
    return np.array([4], np.int32), dist, rng.integers(0, 3, size=(130, N)).astype(np.int16), 2


PATH_CASES = {
    "ragged": _case_ragged,
    "wide_x100": lambda: _case_wide(100, 100),
    "wide_x14": lambda: _case_wide(14, 300),
    "mixed_fallback": _case_mixed,
    "long_n1000": _case_long,
    "n1": _case_short,
}


@pytest.mark.parametrize("case", sorted(PATH_CASES))
@pytest.mark.parametrize("path", [1, 2])
def test_routes_forced_path(binding, path, case):
    tour, dist, dem, Q = PATH_CASES[case]()
    binding.set_route_path(path)
    try:
        for v in ((32, 8, 0, 4), (64, 16, 4, 4)):
            binding.set_route_variant(*v)
            _check(binding, tour, dist, dem, Q, "path %d %s %s" % (path, case, v))
    finally:
        binding.set_route_variant(0)
        binding.set_route_path(0)


def test_routes_ordered_path_many_tiles(binding):
    """n = N = 1000 takes the tour-ordered path by itself: 500 tiles plus a
    ragged one, every scenario's costs, predecessors and cuts checked."""
    inst = W.plain_normal(67, 1000, 64 * 500 + 17, 150)
    tour, dist, dem = _inst_arrays(inst)
    assert binding.routes_workspace_bytes(1000, 1000, dem.shape[0]) >= dem.shape[0] * 1056
    _check(binding, tour, dist, dem, inst.Q, "ordered path n=1000 S=32017")


def test_routes_ordered_path_invalid_inputs(binding):
    rng = np.random.default_rng(66)
    N = n = 300
    dist = W.dist_round(_coords(rng, N))
    tour = (rng.permutation(N) + 1).astype(np.int32)
    dem = rng.integers(1, 10, size=(200, N)).astype(np.int16)
    dem[150, tour[7] - 1] = -3
    binding.set_route_path(2)
    try:
        got = _gpu_routes(binding, tour, dist, dem, 30)
        assert (got["costs"] == oracle.INF32).all() and (got["nroutes"] == -1).all()
        dem[150, tour[7] - 1] = 3
        _check(binding, tour, dist, dem, 30, "ordered path, valid after invalid")
    finally:
        binding.set_route_path(0)


# ----------------------------------------------------------------------------
# degenerate cases
# ----------------------------------------------------------------------------
def test_routes_infeasible_scenarios(binding):
    rng = np.random.default_rng(56)
    N = n = 50
    dist = W.dist_round(_coords(rng, N))
    tour = (rng.permutation(N) + 1).astype(np.int32)
    dem = rng.integers(1, 10, size=(300, N)).astype(np.int16)
    dem[::7, tour[10] - 1] = 45  # position 11 alone exceeds Q = 40 in every 7th scenario
    got, ref = _check(binding, tour, dist, dem, 40, "infeasible")
    assert (got["nroutes"][::7] == 0).all() and (got["costs"][::7] == oracle.INF32).all()
    assert (got["pred"][10:, ::7] == 0xFFFF).all()


def test_routes_one_customer_and_capacity_zero(binding):
    rng = np.random.default_rng(57)
    N = 9
    dist = W.dist_round(_coords(rng, N))
    dem = rng.integers(0, 3, size=(130, N)).astype(np.int16)
    _check(binding, np.array([4], np.int32), dist, dem, 2, "n=1")
    _check(binding, (rng.permutation(N) + 1).astype(np.int32), dist, dem, 0, "Q=0")


def test_routes_empty_tour(binding):
    dist = np.zeros((4, 4), np.int32)
    dem = np.ones((70, 3), np.int16)
    t, d, q = (torch.from_numpy(a).cuda() for a in (np.zeros(0, np.int32), dist, dem))
    out = binding.split_routes_device(t, d, q, 5)
    torch.cuda.synchronize()
    h = out.host()
    assert (h["costs"] == 0).all() and (h["nroutes"] == 0).all()


def test_routes_invalid_inputs_mark_every_scenario(binding):
    rng = np.random.default_rng(58)
    N = n = 30
    dist = W.dist_round(_coords(rng, N))
    tour = (rng.permutation(N) + 1).astype(np.int32)
    dem = rng.integers(1, 10, size=(200, N)).astype(np.int16)
    bad_tour = tour.copy()
    bad_tour[3] = N + 5
    got = _gpu_routes(binding, bad_tour, dist, dem, 30)
    assert (got["costs"] == oracle.INF32).all() and (got["nroutes"] == -1).all()
    neg = dem.copy()
    neg[150, tour[7] - 1] = -3
    got = _gpu_routes(binding, tour, dist, neg, 30)
    assert (got["costs"] == oracle.INF32).all() and (got["nroutes"] == -1).all()
    # the same call with valid inputs afterwards is unaffected
    _check(binding, tour, dist, dem, 30, "valid after invalid")


def test_routes_two_calls_share_a_workspace(binding):
    inst = W.plain_normal(59, 80, 2000, 90)
    tour, dist, dem = _inst_arrays(inst)
    t, d, q = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (tour, dist, dem))
    ws = torch.empty(binding.routes_workspace_bytes(tour.size, dist.shape[0] - 1, dem.shape[0]),
                     dtype=torch.uint8, device="cuda")
    a = binding.split_routes_device(t, d, q, inst.Q, workspace=ws)
    b = binding.split_routes_device(t, d, q, inst.Q + 7, workspace=ws)
    torch.cuda.synchronize()
    ref_a = oracle.split_routes(tour, dist, dem, inst.Q, nthreads=THREADS)
    ref_b = oracle.split_routes(tour, dist, dem, inst.Q + 7, nthreads=THREADS)
    _assert_routes_equal(a.host(), ref_a, "first call")
    _assert_routes_equal(b.host(), ref_b, "second call")
