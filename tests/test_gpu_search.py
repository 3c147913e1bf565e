"""The first-stage candidate search with the GPU evaluator: the same seed
gives the same search as with the CPU oracle as evaluator (the GPU sums are
bit-exact, so every selection matches)."""
import os

import numpy as np
import pytest

import oracle
from paper_2602_05179_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_05179_amd import binding as b
    return b


@pytest.mark.parametrize("n,S,Q", [(30, 700, 50), (120, 3000, 100)])
def test_gpu_search_equals_oracle_search(binding, n, S, Q):
    inst = W.plain_normal(50 + n, n, S, Q)
    tours, lens, dist, dem = W.as_arrays(inst)
    kw = dict(population=16, offspring=48, generations=12, mutation=0.35, seed=11)
    d, q = torch.from_numpy(dist).cuda(), torch.from_numpy(dem).cuda()
    gpu = binding.search(d, q, Q, **kw)

    def ev(t):
        return oracle.split_eval(t.ravel(), np.full(t.shape[0], t.shape[1], np.int32), dist, dem, Q,
                                 nthreads=THREADS)["sums"]

    cpu = binding.search(dist, dem, Q, evaluator=ev, **kw)
    assert np.array_equal(gpu["best_tour"], cpu["best_tour"])
    assert gpu["best_sum"] == cpu["best_sum"] and gpu["candidates"] == cpu["candidates"]
    assert np.array_equal(gpu["trace"][:, 1:], cpu["trace"][:, 1:])
    assert (np.diff(gpu["trace"][:, 2]) <= 0).all()


def test_gpu_search_time_budget(binding):
    inst = W.plain_normal(60, 80, 2000, 90)
    tours, lens, dist, dem = W.as_arrays(inst)
    d, q = torch.from_numpy(dist).cuda(), torch.from_numpy(dem).cuda()
    r = binding.search(d, q, inst.Q, population=32, offspring=128, time_budget_s=1.0, seed=3)
    assert r["trace"][-1, 0] < 10.0 and len(r["trace"]) > 2
    assert r["candidates"] == 32 + 128 * (len(r["trace"]) - 1)
    again = oracle.split_eval(r["best_tour"], np.array([80], np.int32), dist, dem, inst.Q)["sums"][0]
    assert again == r["best_sum"]
