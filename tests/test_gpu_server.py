"""Served form on the GPU: continuous batching under an HBM budget, drained
at tile granularity.

Each request's result must be the same alone and in the mix (exactly: all
results are integers and one IEEE division), and equal to the oracle's.
Both drains are covered (pools of at most 256 customers staged in LDS,
larger pools streamed from the tour-ordered copy), both request forms
(resident instances, requests that bring their own instance), the exact
fallback, admission under a budget that forces queueing, the
reservation's halving on out-of-memory, and concurrent clients."""
import sys
import threading
import time

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


def _instances(seed, count, n_hi=1000, S_hi=20_000):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.integers(1, n_hi + 1)) if k % 5 else int(rng.integers(1, 40))
        S = int(rng.integers(1, S_hi)) if k % 3 else int(rng.integers(1, 200))
        Q = int(rng.choice([80, 150, 300]))
        out.append(W.plain_normal(int(rng.integers(0, 2**31 - 1)), n, S, Q))
    return out


def _ref(inst, tour=None):
    tours = inst.tours if tour is None else np.asarray(tour, np.int32)
    lens = np.array([tours.size], np.int32)
    r = oracle.split_eval(tours, lens, inst.dist, inst.demands, inst.Q, nthreads=8)
    return r["costs"][0], int(r["sums"][0]), float(r["means"][0])


def _same(res, ref, label):
    costs, sm, mn = ref
    assert np.array_equal(res["costs"], costs), label
    assert res["sum"] == sm, label
    assert np.float64(res["mean"]).tobytes() == np.float64(mn).tobytes(), label


def test_alone_equals_mix_equals_oracle(binding):
    insts = _instances(31, 24)
    srv = binding.Server(4 << 30, max_len=1024)
    ids = []
    for inst in insts:
        ids.append(srv.add_instance(inst.dist, inst.demands))
    rng = np.random.default_rng(77)
    # every instance with its own tour and a second, reversed tour
    work = []
    for inst, iid in zip(insts, ids):
        work.append((inst, iid, inst.tours))
        work.append((inst, iid, inst.tours[::-1].copy()))
    alone = []
    for inst, iid, tour in work:
        _say("alone " + inst.name)
        alone.append(srv.wait(srv.submit(iid, tour, inst.Q, inst.S, want_costs=True)))
    _say("mix of %d" % len(work))
    order = rng.permutation(len(work))
    rids = {}
    for k in order:
        inst, iid, tour = work[k]
        rids[k] = srv.submit(iid, tour, inst.Q, inst.S, want_costs=True)
    mix = {k: srv.wait(r) for k, r in rids.items()}
    st = srv.stats()
    srv.close()
    assert st["peak_bytes"] <= st["capacity"]
    assert st["completed"] == 2 * len(work)
    for k, (inst, iid, tour) in enumerate(work):
        ref = _ref(inst, tour)
        _same(alone[k], ref, "alone " + inst.name)
        _same(mix[k], ref, "mix " + inst.name)
        assert mix[k]["latency_s"] > 0


def test_large_pools_at_the_served_scenario_counts(binding):
    """Requests at the top of the served stream's range (S = 10^5 scenarios,
    pools of 300..1000 customers, all three capacities), submitted together
    so both drains and all four queues run at once; every cost, sum and
    mean equals the oracle's."""
    rng = np.random.default_rng(91)
    insts = [W.plain_normal(int(rng.integers(0, 2**31 - 1)), n, 100_000, Q)
             for n, Q in ((1000, 300), (640, 150), (300, 80), (200, 150), (257, 300))]
    srv = binding.Server(8 << 30, max_len=1024)
    ids = [srv.add_instance(i.dist, i.demands) for i in insts]
    rids = [srv.submit(iid, inst.tours, inst.Q, inst.S, want_costs=True) for inst, iid in zip(insts, ids)]
    res = [srv.wait(r) for r in rids]
    srv.close()
    for inst, r in zip(insts, res):
        _say("large " + inst.name)
        _same(r, _ref(inst), "large " + inst.name)


def test_memory_reuse_under_a_deep_backlog(binding):
    """Sixty requests on pools above the LDS path (their tour-ordered copies
    written by the drain waves), submitted at once under a budget that holds
    a few of them: outputs and copies are reused while long-lived drains
    run, and every result still equals the oracle's."""
    rng = np.random.default_rng(93)
    insts = [W.plain_normal(int(rng.integers(0, 2**31 - 1)), int(rng.integers(300, 600)),
                            int(rng.integers(10_000, 30_000)), int(rng.choice([80, 150, 300])))
             for _ in range(6)]
    probe = binding.Server(2 << 30, max_len=1024)
    pids = [probe.add_instance(i.dist, i.demands) for i in insts]
    resident = probe.stats()["bytes_in_use"]
    probe.close()
    srv = binding.Server(resident + (160 << 20), max_len=1024)
    ids = [srv.add_instance(i.dist, i.demands) for i in insts]
    work = []
    for k in range(60):
        j = k % len(insts)
        tour = rng.permutation(insts[j].N).astype(np.int32) + 1
        work.append((j, tour))
    rids = [srv.submit(ids[j], tour, insts[j].Q, insts[j].S, want_costs=True) for j, tour in work]
    res = [srv.wait(r) for r in rids]
    st = srv.stats()
    srv.close()
    assert st["blocked_rounds"] > 0, "the budget should make admission wait"
    for (j, tour), r in zip(work, res):
        _same(r, _ref(insts[j], tour), "reuse " + insts[j].name)


def test_requests_with_their_own_instance(binding):
    insts = _instances(41, 10, n_hi=600, S_hi=8000)
    srv = binding.Server(2 << 30, max_len=1024)
    rids = [srv.submit_copy(inst.tours, inst.dist, inst.demands, inst.Q, want_costs=True) for inst in insts]
    res = [srv.wait(r) for r in rids]
    # an own instance's demands are released once the drains that were
    # running when its request completed have ended (they leave after a
    # short time without work)
    deadline = time.monotonic() + 5.0
    st = srv.stats()
    while st["bytes_in_use"] and time.monotonic() < deadline:
        time.sleep(0.002)
        st = srv.stats()
    srv.close()
    assert st["bytes_in_use"] == 0, "own instances are released after their requests complete"
    for inst, r in zip(insts, res):
        _say("own instance " + inst.name)
        _same(r, _ref(inst), inst.name)


@pytest.mark.parametrize("N", [120, 700])
def test_exact_fallback_tiles(binding, N):
    """Windows past the 64-entry register ring (unit demands, large Q) and
    demands past a byte take the exact path inside the drain."""
    rng = np.random.default_rng(N)
    dist = W.dist_round(W.coords(rng, N))
    tour = (rng.permutation(N) + 1).astype(np.int32)
    dem = rng.integers(1, 12, size=(64 * 7 + 5, N)).astype(np.int16)
    dem[64:128] = 1                                      # windows of ~100 positions at Q = 300
    dem[64 * 3:64 * 4] = rng.integers(200, 300, size=(64, N))  # past a byte, hard capacity 300
    srv = binding.Server(1 << 30, max_len=1024)
    iid = srv.add_instance(dist, dem)
    for Q in (300, 120):
        _say("fallback N=%d Q=%d" % (N, Q))
        r = srv.wait(srv.submit(iid, tour, Q, dem.shape[0], want_costs=True))
        inst = W.Instance(name="fb", tours=tour, lens=np.array([N], np.int32), dist=dist, demands=dem, Q=Q,
                          seed=N)
        _same(r, _ref(inst), "fallback N=%d Q=%d" % (N, Q))
    srv.close()


def test_budget_forces_queueing(binding):
    """A budget that holds about two requests: the rest wait for memory,
    every result is still exact and the arena never exceeds the budget."""
    insts = _instances(32, 8, n_hi=400, S_hi=6000)
    base = binding.Server(1 << 30, max_len=512)
    ids = [base.add_instance(i.dist, i.demands) for i in insts]
    resident = base.stats()["bytes_in_use"]
    peak = 0
    for inst, iid in zip(insts, ids):
        base.wait(base.submit(iid, inst.tours, inst.Q))
        peak = max(peak, base.stats()["peak_bytes"] - resident)
    base.close()
    budget = resident + 2 * peak + (96 << 20)  # fixed structures take part of the reservation
    srv = binding.Server(budget, max_len=512)
    ids = [srv.add_instance(i.dist, i.demands) for i in insts]
    rids = [srv.submit(iid, inst.tours, inst.Q, inst.S, want_costs=True) for inst, iid in zip(insts, ids)]
    res = [srv.wait(r) for r in rids]
    st = srv.stats()
    srv.close()
    assert st["peak_bytes"] <= st["capacity"]
    for inst, r in zip(insts, res):
        _same(r, _ref(inst), "queued " + inst.name)


def test_reservation_halves_on_out_of_memory(binding):
    """The paper's batch loop retries with a smaller batch after an
    out-of-memory error; the server's reservation does the same."""
    binding.debug_fail_allocations(0)
    full = binding.Server(1 << 30, max_len=256)
    cap_full = full.stats()["capacity"]
    full.close()
    binding.debug_fail_allocations(2)
    try:
        srv = binding.Server(1 << 30, max_len=256)
    finally:
        binding.debug_fail_allocations(0)
    cap = srv.stats()["capacity"]
    assert cap < cap_full // 3, (cap, cap_full)
    inst = W.plain_normal(7, 150, 3000, 150)
    iid = srv.add_instance(inst.dist, inst.demands)
    r = srv.wait(srv.submit(iid, inst.tours, inst.Q, inst.S, want_costs=True))
    srv.close()
    _same(r, _ref(inst), "after halving")


def test_concurrent_clients(binding):
    insts = _instances(33, 6, n_hi=300, S_hi=3000)
    srv = binding.Server(1 << 30, max_len=512)
    ids = [srv.add_instance(i.dist, i.demands) for i in insts]
    out = {}
    errors = []

    def client(k):
        try:
            got = []
            for rep in range(4):
                inst, iid = insts[(k + rep) % len(insts)], ids[(k + rep) % len(insts)]
                rid = srv.submit(iid, inst.tours, inst.Q, inst.S, want_costs=True)
                got.append(((k + rep) % len(insts), srv.wait(rid)))
            out[k] = got
        except Exception as e:  # reported below
            errors.append(e)

    threads = [threading.Thread(target=client, args=(k,)) for k in range(6)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    srv.close()
    assert not errors, errors
    refs = [_ref(i) for i in insts]
    for k, got in out.items():
        for idx, r in got:
            _same(r, refs[idx], "client %d" % k)


def test_oversized_request_and_bad_input(binding):
    inst = W.plain_normal(5, 200, 5000, 150)
    srv = binding.Server(1 << 20, max_len=256)  # raised to the 64 MiB floor
    cap = srv.stats()["capacity"]
    big = np.ones((cap // (2 * 200) + 64, 200), np.int16)  # demands past the whole budget
    with pytest.raises(binding.SplitError) as e:
        srv.add_instance(inst.dist, big)
    assert e.value.code == binding.SPLIT_ENOMEM
    with pytest.raises(binding.SplitError) as e:
        srv.submit_copy(inst.tours, inst.dist, big, inst.Q)
    assert e.value.code == binding.SPLIT_ENOMEM
    del big
    srv.close()
    srv = binding.Server(1 << 30, max_len=256)
    iid = srv.add_instance(inst.dist, inst.demands)
    bad = inst.tours.copy()
    bad[3] = 0
    with pytest.raises(binding.SplitError) as e:
        srv.submit(iid, bad, inst.Q)
    assert e.value.code == binding.SPLIT_EINVAL
    bad[3] = 10 ** 6  # an id far past the cost matrix is rejected before it is read
    with pytest.raises(binding.SplitError) as e:
        srv.submit(iid, bad, inst.Q)
    assert e.value.code == binding.SPLIT_EINVAL
    with pytest.raises(binding.SplitError) as e:
        srv.submit(iid + 100, inst.tours, inst.Q)
    assert e.value.code == binding.SPLIT_EINVAL
    long_tour = np.ones(300, np.int32)
    with pytest.raises(binding.SplitError) as e:  # longer than the server's max_len
        srv.submit(iid, long_tour, inst.Q)
    assert e.value.code == binding.SPLIT_EINVAL
    # a negative demand is found on the device and reported at poll
    dem = inst.demands.copy()
    dem[17, inst.tours[5] - 1] = -3
    iid2 = srv.add_instance(inst.dist, dem)
    rid = srv.submit(iid2, inst.tours, inst.Q)
    with pytest.raises(binding.SplitError) as e:
        srv.wait(rid)
    assert e.value.code == binding.SPLIT_EINVAL
    # the server keeps serving after a rejected request
    r = srv.wait(srv.submit(iid, inst.tours, inst.Q, inst.S, want_costs=True))
    _same(r, _ref(inst), "after errors")
    srv.remove_instance(iid)
    srv.remove_instance(iid2)
    assert srv.stats()["instances"] == 0
    srv.close()
