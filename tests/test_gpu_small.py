"""GPU parity of the one-launch form (one short tour, a few thousand
scenarios: tables, recursion, exact fallback and the fold in one workgroup).

Every shape here is checked to take that form (split_eval_path), then its
costs, sums and means are compared element by element and bit for bit with
the CPU oracle, and with the general kernels forced by a schedule override
on the same device inputs.  Inputs the device rejects (ids, cost range, the
int32 guard, lengths, negative demands) are compared with the general
kernels and with the documented result (SPLIT_INF costs, SPLIT_SUM_INVALID,
NaN mean).
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
    yield b
    b.set_schedule(0)


def _default_variant(Q):
    # the built-in default window variant for a capacity
    if Q > 200:
        return (64, 16, 4, 4)
    return (32, 8, 3, 3) if Q > 100 else (32, 6, 3, 3)


def _dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def _eval(binding, dev, Q, max_len):
    t, l, d, q = dev
    out = binding.split_eval_device(t, l, d, q, Q, max_len=max_len)
    torch.cuda.synchronize()
    return dict(costs=out.costs.cpu().numpy(), sums=out.sums.cpu().numpy(),
                means=out.means.cpu().numpy())


def _same(got, ref, label):
    gc, rc = got["costs"], ref["costs"]
    assert gc.shape == rc.shape, label
    bad = np.argwhere(gc != rc)
    assert bad.size == 0, "%s: %d cost mismatches, first at %s: got %d want %d" % (
        label, len(bad), bad[0], gc[tuple(bad[0])], rc[tuple(bad[0])])
    assert np.array_equal(got["sums"], ref["sums"]), (label, got["sums"], ref["sums"])
    assert np.array_equal(got["means"].view(np.int64), ref["means"].view(np.int64)), label


def _one_launch_vs_general(binding, tour, dist, dem, Q, *, max_len=None, lens=None,
                           variant=None, label=""):
    """Evaluates through the one-launch form and through the general kernels
    (same variant, path forced); asserts the one-launch form was taken."""
    tour = np.asarray(tour, np.int32)
    lens = np.array([len(tour)], np.int32) if lens is None else np.asarray(lens, np.int32)
    max_len = int(lens.max()) if max_len is None else int(max_len)
    N, S = dist.shape[0] - 1, dem.shape[0]
    v = variant or _default_variant(Q)
    _say("%s n=%d max_len=%d N=%d S=%d Q=%d variant=%s" % (label, int(lens[0]), max_len, N, S, Q, v))
    dev = _dev(tour, lens, dist, dem)
    try:
        binding.set_schedule(*v, waves=0, path=0)
        assert binding.eval_path(1, max_len, N, S, Q) == binding.PATH_ONE_LAUNCH, label
        one = _eval(binding, dev, Q, max_len)
        binding.set_schedule(*v, waves=0, path=1)
        assert binding.eval_path(1, max_len, N, S, Q) == binding.PATH_TILES, label
        gen = _eval(binding, dev, Q, max_len)
    finally:
        binding.set_schedule(0)
    _same(one, gen, label + " (one launch vs general kernels)")
    return one


def _vs_oracle(binding, tour, dist, dem, Q, label, **kw):
    one = _one_launch_vs_general(binding, tour, dist, dem, Q, label=label, **kw)
    lens = np.array([len(tour)], np.int32)
    ref = oracle.split_eval(np.asarray(tour, np.int32), lens, dist, dem, Q, nthreads=THREADS)
    _same(one, ref, label + " (one launch vs oracle)")
    return one


def _edge_instances():
    rng = np.random.default_rng(300)
    N = 120
    dist = W.dist_round(W.coords(rng, N))
    tour = W.random_tour(rng, N)
    dem = W.demands_uniform(rng, 1000, N, 1, 10)
    out = [("n=1", tour[:1], dist, dem, 10),
           ("whole tour fits (windows past the ring)", tour, dist, dem[:500], 10_000),
           ("window of one", tour, dist, W.demands_uniform(rng, 600, N, 6, 10), 10)]
    d2 = dem.copy()
    d2[5, 7] = 40
    d2[70, :] = 40
    out.append(("some demands over Q", tour, dist, d2, 30))
    for S in (1, 63, 64, 65, 129, 511, 1000, 1024):
        out.append(("S=%d" % S, tour, dist, dem[:S], 30))
    d3 = dem.copy()
    d3[3, 11] = 300
    d3[600, :5] = 32767
    out.append(("demands above one byte", tour, dist, d3, 40_000))
    out.append(("zero demands, Q=0", tour, dist, np.zeros_like(dem), 0))
    ones = np.ones((300, N), np.int16)
    for w in (31, 32, 33, 63, 64, 65):
        out.append(("unit demands, window %d" % w, tour, dist, ones, w))
    asym = rng.integers(0, 1000, size=(N + 1, N + 1)).astype(np.int32)
    out.append(("asymmetric costs", tour, asym, dem, 25))
    # the int32 guard at its limit: 3 * 120 * 1491308 < 2^29 (accepted)
    big = np.full((N + 1, N + 1), 1_491_308, np.int32)
    out.append(("costs at the exactness guard", tour, big, dem[:200], 30))
    return out


@pytest.mark.parametrize("k", range(len(_edge_instances())))
def test_edge_cases_against_oracle(binding, k):
    name, tour, dist, dem, Q = _edge_instances()[k]
    _vs_oracle(binding, tour, dist, dem, Q, name)


def test_smallest_named_workload(binding):
    """The n=20, S=1000, Q=30 workload, device and host forms."""
    inst = W.plain_small(1, S=1000)
    tours, lens, dist, dem = W.as_arrays(inst)
    one = _vs_oracle(binding, tours, dist, dem, inst.Q, "n=20 S=1000 Q=30")
    assert binding.eval_path(1, 20, inst.N, 1000, inst.Q) == binding.PATH_ONE_LAUNCH
    _same(binding.split_eval(tours, lens, dist, dem, inst.Q), one, "host form")


_VARIANTS = [(32, 8, 3, 3), (32, 8, 0, 4), (32, 8, 3, 2), (32, 8, 2, 2), (32, 6, 3, 3),
             (32, 6, 2, 2), (32, 10, 3, 3), (64, 16, 4, 4), (64, 16, 0, 6), (64, 20, 4, 3),
             (64, 12, 6, 2), (64, 24, 4, 4)]


@pytest.mark.parametrize("variant", _VARIANTS)
def test_every_window_variant(binding, variant):
    assert variant in binding.list_variants()
    for Q in (30, 150, 300):
        inst = W.plain_normal(40 + Q, 100, 700, Q)
        tours, _, dist, dem = W.as_arrays(inst)
        _vs_oracle(binding, tours, dist, dem, Q, "n=100 S=700 Q=%d" % Q, variant=variant)


def test_random_shapes(binding):
    rng = np.random.default_rng(301)
    for i in range(12):
        n = int(rng.integers(1, 200))
        tiles_per_wave = max(1, 256 // n)
        S = int(rng.integers(1, min(8 * 64 * tiles_per_wave, 4096) + 1))
        N = int(rng.integers(n, 257))
        Q = int(rng.choice([20, 60, 150, 250]))
        dist = W.dist_round(W.coords(rng, N))
        tour = W.random_tour(rng, N)[:n]
        dem = W.demands_poisson(rng, S, rng.uniform(2, 15, size=N))
        _vs_oracle(binding, tour, dist, dem, Q, "random %d" % i)


def test_size_limits(binding):
    """The boundary shapes of the one-launch form (256 recursion steps per
    wave, pools of 256 customers) against the oracle; the path choice at
    these sizes is checked on the CPU."""
    # the boundary shapes themselves, against the oracle
    rng = np.random.default_rng(302)
    for n, N, S in ((128, 200, 1024), (256, 256, 512), (20, 256, 1000)):
        dist = W.dist_round(W.coords(rng, N))
        tour = W.random_tour(rng, N)[:n]
        dem = W.demands_uniform(rng, S, N, 1, 10)
        _vs_oracle(binding, tour, dist, dem, 100, "limit n=%d N=%d S=%d" % (n, N, S))


def test_empty_tour_and_bounds_from_the_host(binding):
    rng = np.random.default_rng(303)
    N = 50
    dist = W.dist_round(W.coords(rng, N))
    tour = W.random_tour(rng, N)
    dem = W.demands_uniform(rng, 300, N, 1, 10)
    # n = 0 on the device under a host bound of 40: cost 0 everywhere
    one = _one_launch_vs_general(binding, tour[:1], dist, dem, 30, lens=[0], max_len=40,
                                 label="n=0 under max_len=40")
    assert (one["costs"] == 0).all() and one["sums"][0] == 0 and one["means"][0] == 0.0
    # a length above the host bound is rejected on the device
    one = _one_launch_vs_general(binding, tour[:30], dist, dem, 30, lens=[30], max_len=20,
                                 label="n=30 over max_len=20")
    _assert_invalid(binding, one)
    # a tour shorter than the host bound
    got = _one_launch_vs_general(binding, tour[:25], dist, dem, 30, max_len=45,
                                 label="n=25 under max_len=45")
    ref = oracle.split_eval(tour[:25].astype(np.int32), np.array([25], np.int32), dist, dem, 30)
    _same(got, ref, "n=25 under max_len=45 (oracle)")


def _assert_invalid(binding, got):
    assert (got["costs"] == binding.SPLIT_INF).all()
    assert got["sums"][0] == binding.SPLIT_SUM_INVALID and np.isnan(got["means"][0])


def test_inputs_rejected_on_the_device(binding):
    rng = np.random.default_rng(304)
    N = 60
    dist = W.dist_round(W.coords(rng, N))
    tour = W.random_tour(rng, N)
    dem = W.demands_uniform(rng, 700, N, 1, 10)
    cases = []
    t0 = tour.copy()
    t0[17] = 0
    cases.append(("customer id 0", t0, dist, dem))
    t1 = tour.copy()
    t1[0] = N + 1
    cases.append(("customer id N+1 in first position", t1, dist, dem))
    d1 = dist.copy()
    d1[tour[10], tour[11]] = (1 << 24) + 1
    cases.append(("a leg above the cost bound", tour, d1, dem))
    d2 = dist.copy()
    d2[0, tour[-1]] = d2[tour[-1], 0] = -1
    cases.append(("a negative depot leg", tour, d2, dem))
    big = np.full((N + 1, N + 1), 3_000_000, np.int32)
    cases.append(("the exactness guard exceeded", tour, big, dem))
    q1 = dem.copy()
    q1[650, tour[3] - 1] = -2
    cases.append(("a negative demand", tour, dist, q1))
    for name, t, d, q in cases:
        got = _one_launch_vs_general(binding, t, d, q, 30, label=name)
        _assert_invalid(binding, got)


def test_plan_graph_replays(binding):
    """A captured plan of a one-launch shape, replayed as a graph and as
    eager launches in turn, gives the oracle's result every time."""
    inst = W.plain_small(7, S=1000)
    tours, lens, dist, dem = W.as_arrays(inst)
    ref = oracle.split_eval(tours, lens, dist, dem, inst.Q)
    t, l, d, q = _dev(tours, lens, dist, dem)
    plan = binding.Plan(t, l, d, q, inst.Q, int(lens.max()))
    try:
        for r in range(6):
            out = plan.launch() if r % 2 == 0 else plan.launch_eager()
            torch.cuda.synchronize()
            got = dict(costs=out.costs.cpu().numpy(), sums=out.sums.cpu().numpy(),
                       means=out.means.cpu().numpy())
            _same(got, ref, "replay %d" % r)
            torch.zeros(1 << 20, device="cuda").add_(1)  # eager work between replays
            torch.cuda.synchronize()
    finally:
        plan.close()


def test_repeated_calls_reuse_the_workspace(binding):
    """Back-to-back calls on one workspace, the second smaller: no state
    of the first survives into the second."""
    rng = np.random.default_rng(305)
    N = 90
    dist = W.dist_round(W.coords(rng, N))
    tour = W.random_tour(rng, N)
    dem = W.demands_uniform(rng, 1000, N, 1, 12)
    t, l, d, q = _dev(tour, np.array([N], np.int32), dist, dem)
    ws = None
    for n, S in ((90, 1000), (33, 130), (90, 64)):
        l2 = torch.tensor([n], dtype=torch.int32, device="cuda")
        qs = q[:S].contiguous()
        assert binding.eval_path(1, N, N, S, 40) == binding.PATH_ONE_LAUNCH
        out = binding.split_eval_device(t, l2, d, qs, 40, max_len=N, workspace=ws)
        ws = out.workspace
        torch.cuda.synchronize()
        got = dict(costs=out.costs.cpu().numpy(), sums=out.sums.cpu().numpy(),
                   means=out.means.cpu().numpy())
        ref = oracle.split_eval(tour[:n].astype(np.int32), np.array([n], np.int32), dist, dem[:S], 40)
        _same(got, ref, "n=%d S=%d" % (n, S))


def test_tuner_times_the_one_launch_form(binding):
    """The tuner's candidates include the one-launch form (recorded as path
    0); whichever wins, the next evaluation of the shape takes the recorded
    path and equals the oracle."""
    binding.tune_clear()
    try:
        inst = W.plain_small(9, S=1000)
        tours, lens, dist, dem = W.as_arrays(inst)
        t, l, d, q = _dev(tours, lens, dist, dem)
        ms = binding.tune_device(t, l, d, q, inst.Q, reps=5)
        rec = binding.tune_lookup(1, 20, inst.N, inst.S, inst.Q)
        _say("tuned n=20 S=1000 -> %s (%.4f ms)" % (rec, ms))
        assert ms > 0 and rec is not None and rec[5] in (0, 1)
        want = binding.PATH_ONE_LAUNCH if rec[5] == 0 else binding.PATH_TILES
        assert binding.eval_path(1, 20, inst.N, inst.S, inst.Q) == want
        got = _eval(binding, (t, l, d, q), inst.Q, 20)
        _same(got, oracle.split_eval(tours, lens, dist, dem, inst.Q), "after tuning")
    finally:
        binding.tune_clear()


_PLAN_FIRST = r'''
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import oracle
from paper_2602_05179_amd import binding, workloads as W
inst = W.plain_small(11, S=1000)
tours, lens, dist, dem = W.as_arrays(inst)
t, l, d, q = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (tours, lens, dist, dem))
assert binding.eval_path(1, 20, inst.N, inst.S, inst.Q) == binding.PATH_ONE_LAUNCH
plan = binding.Plan(t, l, d, q, inst.Q, 20)   # the process's first evaluation
ref = oracle.split_eval(tours, lens, dist, dem, inst.Q)
for r in range(3):
    out = plan.launch() if r != 1 else plan.launch_eager()
    torch.cuda.synchronize()
    assert np.array_equal(out.costs.cpu().numpy(), ref["costs"]), r
    assert np.array_equal(out.sums.cpu().numpy(), ref["sums"]), r
plan.close()
print("plan-first ok")
'''


def test_plan_as_the_first_evaluation_of_a_process(binding):
    """A fresh process whose first evaluation is a captured plan of a
    one-launch shape: the kernels' one-time set-up happens before the
    capture, and the graph and eager replays equal the oracle."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    _say("plan-first subprocess")
    r = subprocess.run([sys.executable, "-c", _PLAN_FIRST, root], capture_output=True, text=True,
                       timeout=300, cwd=root)
    assert r.returncode == 0 and "plan-first ok" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
