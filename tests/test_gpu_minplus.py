"""GPU parity of the min-plus Bellman update, its backtracking and the
order-up-to inventory transition generator (through the C ABI) against
the numpy oracle.  Bit-exact: values, recorded minimisers, state paths and
transition matrices."""
import sys

import numpy as np
import pytest

from oracle import minplus as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

INF = M.INF


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_05179_amd import binding as b
    return b


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _run(binding, A, J0, shared):
    JT, arg = binding.minplus_forward(_dev(A), _dev(J0), shared=shared)
    path = binding.minplus_backtrack(JT, arg)
    torch.cuda.synchronize()
    return JT.cpu().numpy().astype(np.int64), arg.cpu().numpy().astype(np.int64), \
        path.cpu().numpy().astype(np.int64)


def _compare(binding, A, J0, shared, label):
    _say("%s A%s shared=%d" % (label, A.shape, shared))
    JT, arg, path = _run(binding, A, J0, shared)
    rJT, rarg = M.minplus_forward(A, J0, shared)
    assert np.array_equal(JT, rJT), label
    assert np.array_equal(arg, rarg), label
    assert np.array_equal(path, M.backtrack(rJT, rarg)), label


def test_paper_illustrative_update(binding):
    J = np.array([[0, 1, 3]])
    A = np.array([[[2, 5, INF], [1, INF, INF], [3, 0, INF]]])  # 3 -> 2 states, padded
    JT, arg, _ = _run(binding, A, J, shared=True)
    assert JT[0, :2].tolist() == [2, 3] and JT[0, 2] == INF
    assert arg[0, 0, :2].tolist() == [0, 2]


def test_paper_inventory_example(binding):
    T, B = 2, 1
    demand = _dev(np.ones((T, B)))
    cost = _dev(np.zeros((T, B, 1)))
    cap = _dev(np.full((T, B, 1), 2))
    A = binding.ou_transitions(2, demand, cost, cap, _dev(np.array([5, 1, 0])), 1, 0)
    torch.cuda.synchronize()
    assert A.cpu().numpy()[0, 0].tolist() == [[5, 3, INF], [5, 2, INF], [INF, 1, INF]]
    JT, arg = binding.minplus_forward(A, _dev(np.array([[INF, 0, INF]])), shared=False)
    path = binding.minplus_backtrack(JT, arg)
    torch.cuda.synchronize()
    assert JT.cpu().numpy().tolist() == [[7, 4, INF]]
    assert path.cpu().numpy()[:, 0].tolist() == [1, 1, 1]


@pytest.mark.parametrize("m", [1, 5, 64, 65, 150])
@pytest.mark.parametrize("shared", [True, False])
def test_random_forward(binding, m, shared):
    rng = np.random.default_rng(m * 7 + shared)
    T = 4 if m <= 65 else 2
    B = 37 if shared else 9
    shape = (T, m, m) if shared else (T, B, m, m)
    A = rng.integers(0, 5, size=shape).astype(np.int64)  # small values: many ties
    A[rng.random(shape) < 0.3] = INF
    J0 = rng.integers(0, 10, size=(B, m)).astype(np.int64)
    J0[rng.random((B, m)) < 0.2] = INF
    J0[0] = INF  # a problem with no allowed start
    _compare(binding, A, J0, shared, "random m=%d" % m)


def test_saturation_and_negative_entries(binding):
    A = np.array([[[INF - 5, 1], [INF - 11, INF]]])
    J0 = np.array([[10, 10], [-1, 3]])  # -1 reads as +inf
    JT, _, _ = _run(binding, A, J0, shared=True)
    assert JT.tolist() == [[INF - 1, 11], [INF - 8, INF]]
    rJT, _ = M.minplus_forward(A, np.where(J0 < 0, INF, J0), True)
    assert np.array_equal(JT, rJT)


@pytest.mark.parametrize("seed", range(4))
def test_inventory_generator_and_forward(binding, seed):
    rng = np.random.default_rng(200 + seed)
    T, B, R = int(rng.integers(1, 6)), 53, int(rng.integers(1, 5))
    U = int(rng.integers(1, 12))
    demand = rng.integers(0, U + 2, size=(T, B))
    cost = rng.integers(0, 40, size=(T, B, R))
    cap = rng.integers(0, U + 1, size=(T, B, R))
    h = rng.integers(0, 9, size=U + 1)
    u, rho = int(rng.integers(0, 3)), int(rng.integers(0, 12))
    I0 = rng.integers(0, U + 1, size=B)
    _say("inventory seed=%d T=%d B=%d R=%d U=%d" % (seed, T, B, R, U))
    A = binding.ou_transitions(U, _dev(demand), _dev(cost), _dev(cap), _dev(h), u, rho)
    torch.cuda.synchronize()
    rA = M.ou_transitions(U, demand, cost, cap, h, u, rho)
    assert np.array_equal(A.cpu().numpy().astype(np.int64), rA)
    J0 = np.full((B, U + 1), INF, np.int64)
    J0[np.arange(B), I0] = 0
    JT, arg = binding.minplus_forward(A, _dev(J0), shared=False)
    torch.cuda.synchronize()
    JT = JT.cpu().numpy().astype(np.int64)
    small = [b for b in range(B)][:6]
    brute = M.ou_brute(U, I0[small], demand[:, small], cost[:, small], cap[:, small], h, u, rho)
    assert np.array_equal(JT[small].min(axis=1), brute)
    rJT, rarg = M.minplus_forward(rA, J0, False)
    assert np.array_equal(JT, rJT) and np.array_equal(arg.cpu().numpy(), rarg)


def test_rejects_bad_sizes(binding):
    A = _dev(np.zeros((1, 2, 2)))
    J0 = _dev(np.zeros((3, 2)))
    with pytest.raises(binding.SplitError):
        binding.minplus_forward(A, J0, shared=False)  # A must be [T, B, m, m]
