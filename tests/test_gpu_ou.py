"""GPU parity of the fused order-up-to inventory DP (one launch, no
transition matrices) against the numpy oracle: the generator's definition
followed by the min-plus forward update (App. B, illustrative matrix form).
Bit-exact: J_T, recorded minimisers and the backtracked state paths."""
import sys

import numpy as np
import pytest

from oracle import minplus as M
from paper_2602_05179_amd import workloads as W

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


def _fused(binding, U, demand, cost, cap, h, u, rho, J0, record_arg=True):
    status = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    JT, arg = binding.ou_dp(U, _dev(demand), _dev(cost), _dev(cap), _dev(h), u, rho, _dev(J0),
                            record_arg=record_arg, status=status)
    torch.cuda.synchronize()
    return (JT.cpu().numpy().astype(np.int64), None if arg is None else arg.cpu().numpy().astype(np.int64),
            int(status.item()))


def _check(binding, U, demand, cost, cap, h, u, rho, J0, label):
    _say(label)
    JT, arg, st = _fused(binding, U, demand, cost, cap, h, u, rho, J0)
    rA = M.ou_transitions(U, demand, cost, cap, h, u, rho)
    rJT, rarg = M.minplus_forward(rA, J0, False)
    assert st == 0, label
    assert np.array_equal(JT, rJT), label
    assert np.array_equal(arg, rarg), label
    path = binding.minplus_backtrack(_dev(JT), _dev(arg))
    torch.cuda.synchronize()
    assert np.array_equal(path.cpu().numpy().astype(np.int64), M.backtrack(rJT, rarg)), label


def _random(seed, T, B, R, U, dmax=None, cmax=40, hmax=9, umax=3, rhomax=12, inf_frac=0.0):
    rng = np.random.default_rng(seed)
    demand = rng.integers(0, (U + 3) if dmax is None else dmax + 1, size=(T, B))
    cost = rng.integers(0, cmax, size=(T, B, R))
    cap = rng.integers(-1, U + 2, size=(T, B, R))
    h = rng.integers(0, hmax, size=U + 1)
    u, rho = int(rng.integers(0, umax)), int(rng.integers(0, rhomax))
    J0 = np.full((B, U + 1), INF, np.int64)
    J0[np.arange(B), rng.integers(0, U + 1, size=B)] = 0
    if inf_frac:
        J0 = rng.integers(0, 30, size=(B, U + 1)).astype(np.int64)
        J0[rng.random((B, U + 1)) < inf_frac] = INF
    return demand, cost, cap, h, u, rho, J0


def test_paper_inventory_example(binding):
    # U = 2, two days, demand 1, transport cost q (one option with room),
    # h = (5, 1, 0), start at level 1: J_3 = (7, 4, +inf), deliver both days
    demand = np.ones((2, 1))
    cost = np.zeros((2, 1, 1))
    cap = np.full((2, 1, 1), 2)
    JT, arg, st = _fused(binding, 2, demand, cost, cap, np.array([5, 1, 0]), 1, 0, np.array([[INF, 0, INF]]))
    assert st == 0
    assert JT.tolist() == [[7, 4, INF]]
    assert arg[0, 0].tolist() == [1, 1, -1] and arg[1, 0].tolist() == [1, 1, -1]
    path = binding.minplus_backtrack(_dev(JT), _dev(arg))
    torch.cuda.synchronize()
    assert path.cpu().numpy()[:, 0].tolist() == [1, 1, 1]


@pytest.mark.parametrize("U", [0, 1, 6, 7, 8, 15, 16, 20, 31])
def test_random_levels(binding, U):
    T, B, R = 5, 64 * 3 + 11, 3
    _check(binding, U, *_random(300 + U, T, B, R, U), label="U=%d T=%d B=%d R=%d" % (U, T, B, R))


@pytest.mark.parametrize("R", [1, 2, 8, 9, 23, 64])
def test_route_option_counts(binding, R):
    # R past the options held in flight exercises the in-loop option reads
    _check(binding, 12, *_random(400 + R, 4, 130, R, 12), label="R=%d" % R)


def test_ties_saturation_and_arbitrary_start(binding):
    # tiny costs (many ties: the smallest predecessor must win), huge rho and
    # u (sums saturate at +inf), arbitrary start vectors with +inf entries
    _check(binding, 9, *_random(7, 6, 200, 4, 9, cmax=2, hmax=2), label="ties")
    d, c, k, h, _, _, J0 = _random(8, 3, 100, 4, 9, inf_frac=0.3)
    _check(binding, 9, d, c, k, h, 1 << 30, (1 << 31) - 1, J0, label="saturation")
    d, c, k, h, u, rho, J0 = _random(9, 3, 100, 4, 9, inf_frac=0.5)
    c[...] = INF  # no option is ever usable: only the no-delivery action
    _check(binding, 9, d, c, k, h, u, rho, J0, label="no usable option")


def test_large_demands_and_long_horizon(binding):
    # demands far past U (everything lands on level 0), one day and many days
    _check(binding, 10, *_random(11, 1, 77, 2, 10, dmax=200), label="T=1 big demands")
    _check(binding, 5, *_random(12, 40, 65, 3, 5), label="T=40")


def test_bench_instance_sampled(binding):
    # the benchmarked instance (100 customers x 1000 scenarios, U=20, T=7,
    # R=4): every problem on the GPU, a sample of problems through the oracle
    inst = W.inventory_ou()
    T, B = inst.demand.shape
    m = inst.U + 1
    J0 = np.full((B, m), INF, np.int64)
    J0[np.arange(B), inst.I0] = 0
    _say("bench instance %s" % inst.name)
    JT, arg, st = _fused(binding, inst.U, inst.demand, inst.opt_cost, inst.opt_cap, inst.h, inst.u, inst.rho, J0)
    assert st == 0
    rng = np.random.default_rng(5)
    sample = np.sort(np.concatenate([[0, B - 1], rng.choice(B, 300, replace=False)]))
    rA = M.ou_transitions(inst.U, inst.demand[:, sample], inst.opt_cost[:, sample], inst.opt_cap[:, sample],
                          inst.h, inst.u, inst.rho)
    rJT, rarg = M.minplus_forward(rA, J0[sample], False)
    assert np.array_equal(JT[sample], rJT)
    assert np.array_equal(arg[:, sample], rarg)


def test_without_minimisers(binding):
    d, c, k, h, u, rho, J0 = _random(13, 4, 90, 3, 7)
    JT, arg, st = _fused(binding, 7, d, c, k, h, u, rho, J0, record_arg=False)
    assert arg is None and st == 0
    rJT, _ = M.minplus_forward(M.ou_transitions(7, d, c, k, h, u, rho), J0, False)
    assert np.array_equal(JT, rJT)


@pytest.mark.parametrize("what", ["demand", "cost", "h"])
def test_status_reports_negative_inputs(binding, what):
    d, c, k, h, u, rho, J0 = _random(14, 3, 70, 2, 5)
    if what == "demand":
        d[1, 65] = -3
    elif what == "cost":
        c[2, 3, 1] = -1
    else:
        h[4] = -2
    _, _, st = _fused(binding, 5, d, c, k, h, u, rho, J0)
    assert st == 1, what


def test_rejects_bad_sizes(binding):
    d, c, k, h, u, rho, J0 = _random(15, 2, 10, 2, 5)
    with pytest.raises(binding.SplitError):
        binding.ou_dp(5, _dev(d), _dev(c), _dev(k), _dev(h), u, rho, _dev(J0[:, :5]))
    with pytest.raises(binding.SplitError):  # U past the fused kernel's 32 levels
        z = np.zeros((2, 10, 2))
        binding.ou_dp(32, _dev(d), _dev(z), _dev(z), _dev(np.zeros(33)), 0, 0, _dev(np.zeros((10, 33))))
