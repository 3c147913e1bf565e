"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every comparison is exact: per-scenario int32 costs element by element, the
int64 sums, and the float64 means bit for bit (both sides divide the same
int64 by the same S in one IEEE division).
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


def _to_dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def _device_eval(binding, tours, lens, dist, dem, Q, max_len=None):
    t, l, d, q = _to_dev(tours, lens, dist, dem)
    out = binding.split_eval_device(t, l, d, q, Q, max_len=max_len)
    torch.cuda.synchronize()
    return dict(costs=out.costs.cpu().numpy(), sums=out.sums.cpu().numpy(), means=out.means.cpu().numpy())


def _assert_same(got, ref, label=""):
    gc, rc = got["costs"], ref["costs"]
    assert gc.shape == rc.shape, label
    bad = np.argwhere(gc != rc)
    assert bad.size == 0, "%s: %d cost mismatches, first at %s: got %d want %d" % (
        label, len(bad), bad[0], gc[tuple(bad[0])], rc[tuple(bad[0])])
    assert np.array_equal(got["sums"], ref["sums"]), label
    assert np.array_equal(got["means"].view(np.int64), ref["means"].view(np.int64)), label


def _run_both(binding, inst, label=None, host_form=False):
    label = label or inst.name
    tours, lens, dist, dem = W.as_arrays(inst)
    _say("%s seed=%d N=%d S=%d T=%d" % (label, inst.seed, inst.N, inst.S, inst.num_tours))
    got = _device_eval(binding, tours, lens, dist, dem, inst.Q)
    ref = oracle.split_eval(tours, lens, dist, dem, inst.Q, nthreads=THREADS)
    _assert_same(got, ref, label)
    if host_form:
        _assert_same(binding.split_eval(tours, lens, dist, dem, inst.Q), ref, label + " (host form)")
    return got, ref


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------
def test_plain_small(binding):
    _run_both(binding, W.plain_small(1, S=1000), host_form=True)


def test_plain_medium(binding):
    _run_both(binding, W.plain_medium(2, S=100_000), host_form=True)


def test_paper_scale_full(binding):
    """n=200, S=10^6, Q=150: every scenario against the oracle."""
    _run_both(binding, W.plain_paper_scale(3, S=1_000_000))


@pytest.mark.parametrize("waves", [0, 1, 2, 8])
def test_batched_tours_per_workgroup(binding, waves):
    """Tours sharing a staged tile: any grouping gives the oracle's results."""
    inst = W.batched_ragged(12, num_tours=37, S=1500)
    binding.set_schedule(32, 8, 0, 4, waves, 1)
    try:
        _run_both(binding, inst, label="%s waves=%d" % (inst.name, waves))
    finally:
        binding.set_schedule(0)


def test_batched_ragged_and_equal_to_plain(binding):
    inst = W.batched_ragged(4)
    got, ref = _run_both(binding, inst)
    # the ragged batch equals one launch per tour
    tours, lens, dist, dem = W.as_arrays(inst)
    off = 0
    for t in range(0, inst.num_tours, 37):
        n = int(lens[t])
        off = int(lens[:t].sum())
        one = _device_eval(binding, tours[off:off + n], lens[t:t + 1], dist, dem, inst.Q)
        assert np.array_equal(one["costs"][0], got["costs"][t])
        assert one["sums"][0] == got["sums"][t]


def test_batched_by_length_ties_empty_and_invalid(binding):
    """Ragged batch taken in decreasing length: equal lengths, empty tours
    and an invalid tour in the batch; every valid tour equals the oracle."""
    rng = np.random.default_rng(21)
    N, S, Q = 60, 700, 40
    dist = W.dist_round(W.coords(rng, N))
    dem = W.demands_poisson(rng, S, rng.uniform(2.0, 9.0, size=N))
    sizes = [30, 30, 0, 50, 30, 50, 10, 60, 0, 30, 45, 45, 7, 60, 30, 12, 50, 1, 30, 25]
    tours_list = [W.random_tour(rng, N)[:k] if k else np.zeros(0, np.int32) for k in sizes]
    lens = np.array(sizes, np.int32)
    tours = np.concatenate(tours_list).astype(np.int32)
    bad = int(lens[:5].sum()) + 3  # tour 5 gets an invalid customer id
    tours_bad = tours.copy()
    tours_bad[bad] = N + 1
    got = _device_eval(binding, tours_bad, lens, dist, dem, Q)
    ref = oracle.split_eval(tours, lens, dist, dem, Q, nthreads=THREADS)
    for t in range(len(sizes)):
        if t == 5:
            assert got["sums"][t] == binding.SPLIT_SUM_INVALID
            assert (got["costs"][t] == binding.SPLIT_INF).all()
        else:
            assert np.array_equal(got["costs"][t], ref["costs"][t]), t
            assert got["sums"][t] == ref["sums"][t], t


# ----------------------------------------------------------------------------
# edge cases
# ----------------------------------------------------------------------------
def _inst(name, tours_list, dist, dem, Q, seed=0):
    lens = np.array([len(t) for t in tours_list], np.int32)
    tours = np.concatenate([np.asarray(t, np.int32) for t in tours_list]) if len(tours_list) else np.zeros(0, np.int32)
    return W.Instance(name, tours.astype(np.int32), lens, dist.astype(np.int32), dem.astype(np.int16), int(Q), seed)


def _edge_instances():
    rng = np.random.default_rng(100)
    out = []
    N = 120
    dist = W.dist_round(W.coords(rng, N))
    tour = W.random_tour(rng, N)
    dem = W.demands_uniform(rng, 200, N, 1, 10)
    out.append(_inst("n=1", [tour[:1]], dist, dem, 10))
    out.append(_inst("whole tour fits (window past the ring)", [tour], dist, dem, 10_000))
    out.append(_inst("window of one (every pair over Q)", [tour], dist, W.demands_uniform(rng, 200, N, 6, 10), 10))
    d2 = dem.copy()
    d2[5, 7] = 40
    d2[70, :] = 40
    out.append(_inst("some demands over Q", [tour], dist, d2, 30))
    for S in (1, 63, 65, 129):
        out.append(_inst("S=%d" % S, [tour], dist, dem[:S], 30))
    d3 = dem.copy()
    d3[3, 11] = 300
    d3[130, :5] = 32767
    out.append(_inst("demands above one byte", [tour], dist, d3, 40_000))
    out.append(_inst("zero demands, Q=0", [tour], dist, np.zeros_like(dem), 0))
    out.append(_inst("ragged lengths at ring boundaries",
                     [tour[:0], tour[:1], tour[:31], tour[:32], tour[:33], tour[:64], tour[:65], tour[:120]],
                     dist, dem, 30))
    # windows of exactly 31, 32, 33 and 63, 64, 65 customers (unit demands)
    ones = np.ones((130, N), np.int16)
    for w in (31, 32, 33, 63, 64, 65):
        out.append(_inst("unit demands, window %d" % w, [tour], dist, ones, w))
    asym = rng.integers(0, 1000, size=(N + 1, N + 1)).astype(np.int32)
    out.append(_inst("asymmetric costs", [tour, tour[::-1].copy()], asym, dem, 25))
    return out


# one variant without and one with a second head group, per ring length
_EDGE_VARIANTS = [(32, 8, 0, 4), (32, 8, 3, 2), (64, 16, 0, 6), (64, 12, 6, 2)]


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("variant", _EDGE_VARIANTS)
@pytest.mark.parametrize("k", range(len(_edge_instances())))
def test_edge_cases(binding, k, variant, path):
    inst = _edge_instances()[k]
    binding.set_schedule(*variant, waves=0, path=path)
    try:
        _run_both(binding, inst, label="%s variant=%s path=%d" % (inst.name, variant, path),
                  host_form=True)
    finally:
        binding.set_schedule(0)


@pytest.mark.parametrize("Q", [80, 150, 300])
@pytest.mark.parametrize("path", [0, 1, 2])
def test_served_shapes_both_paths(binding, Q, path):
    """n=1000 requests (the served mix): LDS-staged and tour-ordered paths."""
    inst = W.plain_normal(20 + Q, 1000, 3000, Q)
    if path:
        v = (64, 16, 0, 6) if Q > 200 else (32, 8, 0, 4)
        binding.set_schedule(*v, waves=0, path=path)
    try:
        _run_both(binding, inst, label="%s path=%d" % (inst.name, path))
    finally:
        binding.set_schedule(0)


def test_batched_ordered_path(binding):
    inst = W.batched_ragged(13, num_tours=9, S=700)
    binding.set_schedule(32, 8, 0, 4, 0, 2)
    try:
        _run_both(binding, inst, label=inst.name + " ordered")
    finally:
        binding.set_schedule(0)


def test_every_schedule_on_paper_shape(binding):
    """All compiled schedules give identical results (n=200, Q=150 shape)."""
    inst = W.plain_paper_scale(11, S=20_000)
    tours, lens, dist, dem = W.as_arrays(inst)
    ref = oracle.split_eval(tours, lens, dist, dem, inst.Q, nthreads=THREADS)
    assert binding.SCHEDULES
    for sched in binding.SCHEDULES:
        for path in (1, 2):
            _say("schedule %s path %d" % (sched, path))
            binding.set_schedule(*sched, waves=0, path=path)
            try:
                _assert_same(_device_eval(binding, tours, lens, dist, dem, inst.Q), ref,
                             "schedule %s path %d" % (sched, path))
            finally:
                binding.set_schedule(0)


def test_large_customer_pool_beyond_lds(binding):
    """64 x N demand bytes above the LDS limit: every tile takes the exact fallback."""
    rng = np.random.default_rng(101)
    N = 3000
    dist = W.dist_round(W.coords(rng, N))
    tours = [W.random_tour(rng, N)[:150], W.random_tour(rng, N)[:90]]
    dem = W.demands_uniform(rng, 70, N, 1, 12)
    _run_both(binding, _inst("N=3000 pool", tours, dist, dem, 50))


def test_random_small_instances(binding):
    rng = np.random.default_rng(102)
    for trial in range(40):
        N = int(rng.integers(1, 90))
        T = int(rng.integers(1, 5))
        S = int(rng.integers(1, 300))
        dist = W.dist_round(W.coords(rng, N)) if trial % 3 else rng.integers(0, 300, (N + 1, N + 1))
        tours = [W.random_tour(rng, N)[:int(rng.integers(0, N + 1))] for _ in range(T)]
        hi = int(rng.integers(1, 30))
        dem = rng.integers(0, hi + 1, size=(S, N)).astype(np.int16)
        Q = int(rng.integers(0, 4 * hi + 2))
        _run_both(binding, _inst("random trial %d" % trial, tours, np.asarray(dist), dem, Q, seed=trial))


# ----------------------------------------------------------------------------
# device-side validation
# ----------------------------------------------------------------------------
def test_device_form_flags_invalid_tours(binding):
    inst = W.plain_small(5, S=100)
    tours, lens, dist, dem = W.as_arrays(inst)
    tours2 = np.concatenate([tours, tours]).astype(np.int32)
    tours2[25] = 0  # second tour, invalid id
    got = _device_eval(binding, tours2, np.array([20, 20], np.int32), dist, dem, inst.Q)
    ref = oracle.split_eval(tours, lens, dist, dem, inst.Q)
    assert np.array_equal(got["costs"][0], ref["costs"][0]) and got["sums"][0] == ref["sums"][0]
    assert got["sums"][1] == binding.SPLIT_SUM_INVALID and np.isnan(got["means"][1])
    assert (got["costs"][1] == binding.SPLIT_INF).all()


def test_negative_demand_is_rejected(binding):
    inst = W.plain_small(6, S=100)
    tours, lens, dist, dem = W.as_arrays(inst)
    dem = dem.copy()
    dem[50, 3] = -2
    with pytest.raises(binding.SplitError) as e:
        binding.split_eval(tours, lens, dist, dem, inst.Q)
    assert e.value.code == binding.SPLIT_EINVAL
    got = _device_eval(binding, tours, lens, dist, dem, inst.Q)
    assert got["sums"][0] == binding.SPLIT_SUM_INVALID


# ----------------------------------------------------------------------------
# graphs, cell counts, determinism
# ----------------------------------------------------------------------------
def test_plan_graph_replays_match_eager(binding):
    inst = W.batched_ragged(7, num_tours=24, S=3000)
    tours, lens, dist, dem = W.as_arrays(inst)
    t, l, d, q = _to_dev(tours, lens, dist, dem)
    plan = binding.Plan(t, l, d, q, inst.Q, max_len=400)
    rng = np.random.default_rng(8)
    for rep in range(6):
        _say("plan replay %d" % rep)
        if rep:
            # new candidate tours of the same lengths (the search pattern)
            new = []
            for k in range(inst.num_tours):
                new.append(W.two_opt_perturb(rng, inst.tour(k), 5))
            tours = np.concatenate(new).astype(np.int32)
            t.copy_(torch.from_numpy(tours))
        # graph replays and eager replays of the plan in turn
        plan.launch() if rep % 2 == 0 else plan.launch_eager()
        torch.cuda.synchronize()
        got = dict(costs=plan.out.costs.cpu().numpy(), sums=plan.out.sums.cpu().numpy(),
                   means=plan.out.means.cpu().numpy())
        eager = _device_eval(binding, tours, lens, dist, dem, inst.Q)
        _assert_same(got, eager, "replay %d vs eager" % rep)
        ref = oracle.split_eval(tours, lens, dist, dem, inst.Q, nthreads=THREADS)
        _assert_same(got, ref, "replay %d vs oracle" % rep)
    plan.close()


def test_cell_counter_matches_oracle(binding):
    for inst in (W.plain_medium(2, S=20_000), W.batched_ragged(4, num_tours=16, S=2000)):
        tours, lens, dist, dem = W.as_arrays(inst)
        t, l, q = _to_dev(tours, lens, dem)
        cells = binding.split_count_cells_device(t, l, q, inst.N, inst.Q).cpu().numpy()
        ref = oracle.split_eval(tours, lens, dist, dem, inst.Q, nthreads=THREADS)
        assert np.array_equal(cells, ref["cells"])


def test_repeated_runs_are_bit_identical(binding):
    inst = W.plain_medium(9, S=50_000)
    tours, lens, dist, dem = W.as_arrays(inst)
    a = _device_eval(binding, tours, lens, dist, dem, inst.Q)
    b = _device_eval(binding, tours, lens, dist, dem, inst.Q)
    _assert_same(a, b, "repeat")


def test_tuner_records_a_parity_gated_schedule(binding):
    binding.tune_clear()
    for inst in (W.plain_paper_scale(14, S=30_000), W.batched_ragged(15, num_tours=20, S=2000)):
        tours, lens, dist, dem = W.as_arrays(inst)
        t, l, d, q = _to_dev(tours, lens, dist, dem)
        ms = binding.tune_device(t, l, d, q, inst.Q, reps=2)
        assert ms > 0
        rec = binding.tune_lookup(inst.num_tours, int(lens.max()), inst.N, inst.S, inst.Q)
        assert rec is not None and rec[5] in (1, 2)
        _say("tuned %s -> %s (%.3f ms)" % (inst.name, rec, ms))
        # the next evaluation in this bucket runs the tuned schedule
        _run_both(binding, inst, label=inst.name + " tuned")
    binding.tune_clear()


def test_valu_probe_reports_a_plausible_rate(binding):
    """The roofline reference kernel: an int32 VALU rate within the device's range."""
    rate = binding.probe_valu_peak()
    _say("measured VALU rate %.3e lane-ops/s" % rate)
    # 256 CUs x 64 lanes x 2.4 GHz = 3.9e13 at most; a healthy device is far above 1e12
    assert 1e12 < rate < 6e13
