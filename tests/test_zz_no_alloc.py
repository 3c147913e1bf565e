"""The allocation-free entry point (scratch in a fixed device array):
through the C ABI, its results equal split_eval_device's on the same
inputs, on two calls in a row, the second with a smaller input (the array
keeps the first call's contents; the kernels clear what must start at
zero)."""
import ctypes
import sys

import numpy as np
import pytest

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


def _noalloc(binding, t, l, d, q, T, max_len, N, S, Q):
    costs = torch.empty(T * S, dtype=torch.int32, device="cuda")
    sums = torch.empty(T, dtype=torch.int64, device="cuda")
    means = torch.empty(T, dtype=torch.float64, device="cuda")
    P = ctypes.c_void_p
    rc = binding.lib.split_eval_device_noalloc(
        P(t.data_ptr()), P(l.data_ptr()), T, max_len, P(d.data_ptr()), N, P(q.data_ptr()), S, Q,
        P(costs.data_ptr()), P(sums.data_ptr()), P(means.data_ptr()),
        P(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, binding.last_error()
    torch.cuda.synchronize()
    return costs.cpu().numpy().reshape(T, S), sums.cpu().numpy(), means.cpu().numpy()


def _cases():
    big = W.batched_ragged(11, num_tours=24, S=3000, n_lo=50, n_hi=400)   # several tours, ragged lengths
    small = W.plain_normal(12, 90, 64 * 5 + 17, 100)                # one tour, ragged last tile
    return big, small


def test_noalloc_equals_device_form_twice(binding):
    for inst in _cases():
        _say("noalloc " + inst.name)
        tours, lens, dist, dem = W.as_arrays(inst)
        t, l, d, q = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (tours, lens, dist, dem))
        ref = binding.split_eval_device(t, l, d, q, inst.Q)
        torch.cuda.synchronize()
        got = _noalloc(binding, t, l, d, q, inst.num_tours, int(lens.max()), inst.N, inst.S, inst.Q)
        assert np.array_equal(got[0], ref.costs.cpu().numpy().reshape(inst.num_tours, inst.S)), inst.name
        assert np.array_equal(got[1], ref.sums.cpu().numpy()), inst.name
        assert got[2].tobytes() == ref.means.cpu().numpy().tobytes(), inst.name


def test_noalloc_rejects_sizes_past_the_array(binding):
    # rejected on the host before any device work: the pointers are never used
    P = ctypes.c_void_p
    fake = P(256)
    assert binding.noalloc_scratch_bytes() == 32 << 20
    rc = binding.lib.split_eval_device_noalloc(fake, fake, 64, 4000, fake, 4000, fake, 1_000_000, 150,
                                               fake, fake, fake, None)
    assert rc == binding.SPLIT_EINVAL and "scratch" in binding.last_error()
