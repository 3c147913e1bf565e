"""C-ABI checks that need no GPU: the library loads, exports every symbol
the public header declares, and rejects host-checkable bad arguments before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2602_05179_amd import binding
from paper_2602_05179_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(split_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_expected_entry_points():
    decl = _declared_functions()
    assert "split_eval" in decl and "split_eval_device" in decl
    assert set(decl) == set(binding.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_workspace_size_is_positive_and_monotone():
    a = binding.workspace_bytes(1, 200, 200, 1_000_000, 150)
    b = binding.workspace_bytes(2, 200, 200, 1_000_000, 150)
    c = binding.workspace_bytes(1, 400, 200, 1_000_000, 150)
    assert 0 < a < b and a < c
    assert binding.workspace_bytes(0, 10, 10, 10, 5) == 0
    # a large pool with one tour takes the ordered path: room for the tour-ordered copy
    big = binding.workspace_bytes(1, 1000, 1000, 100_000, 150)
    assert big >= 100_000 * 1000


def test_tuning_table_save_load_roundtrip(tmp_path):
    binding.tune_clear()
    assert binding.tune_lookup(1, 200, 200, 1_000_000, 150) is None
    f = tmp_path / "tune.txt"
    # a table written by hand in the documented text format
    from paper_2602_05179_amd import binding as b
    import ctypes
    key = (0, 7, 7, 9, 7)  # one tour, n~200, N~200, S~1e6, Q~150
    f.write_text("# tours len pool scen cap -> ring first group every waves path\n"
                 "%d %d %d %d %d 32 8 3 2 1 1\n" % key)
    b.tune_load(f)
    assert b.tune_lookup(1, 200, 200, 1_000_000, 150) == (32, 8, 3, 2, 1, 1)
    g = tmp_path / "tune2.txt"
    b.tune_save(g)
    b.tune_clear()
    assert b.tune_lookup(1, 200, 200, 1_000_000, 150) is None
    b.tune_load(g)
    assert b.tune_lookup(1, 200, 200, 1_000_000, 150) == (32, 8, 3, 2, 1, 1)
    b.tune_clear()
    bad = tmp_path / "bad.txt"
    bad.write_text("0 7 7 9 7 33 8 3 3 1 1\n")
    with pytest.raises(b.SplitError):
        b.tune_load(bad)
    del ctypes


def _small():
    inst = W.plain_small(1, S=64)
    return W.as_arrays(inst) + (inst.Q,)


@pytest.mark.parametrize("mutate, msg", [
    (lambda a: a.update(Q=-1), "Q must be"),
    (lambda a: a["tours"].__setitem__(0, 0), "outside [1"),
    (lambda a: a["tours"].__setitem__(3, 99), "outside [1"),
    # a huge id at a middle position is rejected before it indexes the cost matrix
    (lambda a: a["tours"].__setitem__(7, 1 << 30), "outside [1"),
    (lambda a: a["tours"].__setitem__(11, -(1 << 30)), "outside [1"),
    (lambda a: a["dist"].__setitem__((0, a["tours"][0]), -5), "travel cost"),
    (lambda a: a["dist"].__setitem__((a["tours"][2], a["tours"][3]), 1 << 25), "travel cost"),
])
def test_host_form_rejects_bad_arguments_before_device_work(mutate, msg):
    tours, lens, dist, dem, Q = _small()
    args = dict(tours=tours.copy(), lens=lens, dist=dist.copy(), demands=dem, Q=Q)
    mutate(args)
    with pytest.raises(binding.SplitError) as e:
        binding.split_eval(**args)
    assert e.value.code == binding.SPLIT_EINVAL
    assert msg in str(e.value)


def test_exactness_guard_is_enforced():
    tours, lens, dist, dem, Q = _small()
    big = dist.copy()
    big[big > 0] = 1 << 24  # 3 * 20 * 2^24 >= 2^29
    with pytest.raises(binding.SplitError) as e:
        binding.split_eval(tours, lens, big, dem, Q)
    assert e.value.code == binding.SPLIT_EINVAL and "guard" in str(e.value)


def test_device_form_rejects_bad_scalars_before_device_work():
    P = ctypes.c_void_p
    fake = P(256)
    for T, N, S, Q, maxlen in ((0, 5, 10, 3, 5), (1, 0, 10, 3, 5), (1, 5, 0, 3, 5), (1, 5, 10, -2, 5),
                               (1, 5, 10, 3, 70000)):
        rc = binding.lib.split_eval_device(fake, fake, T, maxlen, fake, N, fake, S, Q, fake, fake, fake, fake,
                                           1 << 20, None)
        assert rc == binding.SPLIT_EINVAL, (T, N, S, Q, maxlen)
    # misaligned demands and too-small workspace
    rc = binding.lib.split_eval_device(fake, fake, 1, 5, fake, 5, P(258), 10, 3, fake, fake, fake, fake, 1 << 20,
                                       None)
    assert rc == binding.SPLIT_EINVAL and "aligned" in binding.last_error()
    rc = binding.lib.split_eval_device(fake, fake, 1, 5, fake, 5, fake, 10, 3, fake, fake, fake, fake, 16, None)
    assert rc == binding.SPLIT_EINVAL and "workspace" in binding.last_error()


def test_shape_mismatch_is_rejected_in_the_binding():
    tours, lens, dist, dem, Q = _small()
    with pytest.raises(binding.SplitError):
        binding.split_eval(tours, lens, dist, np.zeros((4, 3), np.int16), Q)


def test_window_variants_listed_and_validated():
    """The compiled variants are listed; set_schedule accepts exactly those."""
    vs = binding.list_variants()
    assert vs and all(len(v) == 4 for v in vs)
    assert {v[0] for v in vs} == {32, 64}
    for ring, first, group, every in vs:
        assert 2 <= first < ring and group >= 0 and every >= 1
    try:
        for v in vs:
            binding.set_schedule(*v, waves=0, path=1)
        bad = (32, 9, 0, 4) if (32, 9, 0, 4) not in vs else (32, 31, 31, 31)
        with pytest.raises(binding.SplitError):
            binding.set_schedule(*bad)
        with pytest.raises(binding.SplitError):
            binding.set_schedule(*vs[0], waves=3)
        with pytest.raises(binding.SplitError):
            binding.set_schedule(*vs[0], path=3)
    finally:
        binding.set_schedule(0)


def test_route_variants_listed_and_validated():
    vs = binding.list_route_variants()
    assert vs and all(len(v) == 4 for v in vs)
    assert {v[0] for v in vs} == {32, 64}
    assert set(vs) <= set(binding.list_variants())  # each is a window variant of the evaluator
    try:
        for v in vs:
            binding.set_route_variant(*v)
        with pytest.raises(binding.SplitError):
            binding.set_route_variant(32, 5, 0, 3)
        with pytest.raises(binding.SplitError):
            binding.set_route_variant(48, 8, 3, 3)
    finally:
        binding.set_route_variant(0)


def test_routes_workspace_size():
    a = binding.routes_workspace_bytes(200, 200, 1_000_000)
    b = binding.routes_workspace_bytes(400, 400, 1_000_000)
    assert 0 < a < b
    assert binding.routes_workspace_bytes(0, 5, 10) > 0
    assert binding.routes_workspace_bytes(-1, 5, 10) == 0
    assert binding.routes_workspace_bytes(70000, 5, 10) == 0


def test_route_path_setting_and_workspace():
    """The ordered path adds the tour-ordered copy (S rows of n rounded up
    to 32 plus 32 bytes) to the workspace; the LDS path does not; an
    impossible ordered path (64 x N bytes past the LDS) falls back."""
    n, N, S = 1000, 1000, 200_000
    pitch = (n + 31) // 32 * 32 + 32
    try:
        binding.set_route_path(binding.ROUTE_PATH_LDS)
        lds = binding.routes_workspace_bytes(n, N, S)
        binding.set_route_path(binding.ROUTE_PATH_ORDERED)
        ordered = binding.routes_workspace_bytes(n, N, S)
        assert ordered - lds >= S * pitch
        assert binding.routes_workspace_bytes(80, 3000, S) < S * 80  # no copy possible
        binding.set_route_path(binding.ROUTE_PATH_AUTO)
        assert binding.routes_workspace_bytes(n, N, S) == ordered   # long tour, large pool
        assert binding.routes_workspace_bytes(200, 200, S) < S * 200  # 12.8 KB tiles stay in LDS
        assert binding.routes_workspace_bytes(300, 300, S) < S * 300  # 19.2 KB too
        assert binding.routes_workspace_bytes(200, 1000, S) >= S * 224  # part of a pool: streamed
        for bad in (-1, 3):
            with pytest.raises(binding.SplitError):
                binding.set_route_path(bad)
    finally:
        binding.set_route_path(0)


def test_variant_path_setting_and_workspace():
    n, N, S = 1000, 1000, 100_000
    pitch = (n + 31) // 32 * 32 + 32
    try:
        binding.set_variant_path(1)
        lds = binding.variant_workspace_bytes(n, N, S, 5)
        binding.set_variant_path(2)
        assert binding.variant_workspace_bytes(n, N, S, 5) - lds >= S * pitch
        binding.set_variant_path(0)
        assert binding.variant_workspace_bytes(n, N, S, 5) - lds >= S * pitch
        assert binding.variant_workspace_bytes(200, 200, S, 0) < S * 200
        for bad in (-1, 3):
            with pytest.raises(binding.SplitError):
                binding.set_variant_path(bad)
    finally:
        binding.set_variant_path(0)


def test_routes_device_form_rejects_bad_arguments_before_device_work():
    P = ctypes.c_void_p
    fake = P(256)
    f = binding.lib.split_routes_device
    for n, N, S, Q in ((5, 0, 10, 3), (5, 5, 0, 3), (5, 5, 10, -2), (70000, 5, 10, 3), (-1, 5, 10, 3)):
        rc = f(fake, n, fake, N, fake, S, Q, fake, fake, fake, fake, fake, 1 << 20, None)
        assert rc == binding.SPLIT_EINVAL, (n, N, S, Q)
    rc = f(fake, 5, fake, 5, P(258), 10, 3, fake, fake, fake, fake, fake, 1 << 20, None)
    assert rc == binding.SPLIT_EINVAL and "aligned" in binding.last_error()
    rc = f(fake, 5, fake, 5, fake, 10, 3, fake, fake, fake, fake, fake, 16, None)
    assert rc == binding.SPLIT_EINVAL and "workspace" in binding.last_error()
    rc = f(fake, 5, fake, 5, fake, 10, 3, fake, None, fake, fake, fake, 1 << 20, None)
    assert rc == binding.SPLIT_EINVAL and "null" in binding.last_error()
    rc = f(fake, 5, fake, 5, fake, 10, 3, fake, fake, fake, fake, P(300), 1 << 20, None)
    assert rc == binding.SPLIT_EINVAL and "aligned" in binding.last_error()


def test_values_device_form_rejects_bad_arguments_before_device_work():
    P = ctypes.c_void_p
    fake = P(256)
    f = binding.lib.split_values_device
    for n, N, S, Q in ((5, 0, 10, 3), (5, 5, 0, 3), (5, 5, 10, -2), (70000, 5, 10, 3), (-1, 5, 10, 3)):
        rc = f(fake, n, fake, N, fake, S, Q, fake, fake, fake, 1 << 20, None)
        assert rc == binding.SPLIT_EINVAL, (n, N, S, Q)
    rc = f(fake, 5, fake, 5, fake, 10, 3, fake, fake, fake, 16, None)
    assert rc == binding.SPLIT_EINVAL and "workspace" in binding.last_error()
    rc = f(fake, 5, fake, 5, fake, 10, 3, None, fake, fake, 1 << 20, None)
    assert rc == binding.SPLIT_EINVAL and "null" in binding.last_error()
    rc = f(fake, 5, fake, 5, fake, 10, 3, fake, None, fake, 1 << 20, None)
    assert rc == binding.SPLIT_EINVAL and "null" in binding.last_error()
    rc = f(fake, 5, fake, 5, fake, 10, 3, fake, fake, P(300), 1 << 20, None)
    assert rc == binding.SPLIT_EINVAL and "aligned" in binding.last_error()
    assert binding.lib.split_values_workspace_bytes(-1, 5, 10) == 0
    assert binding.lib.split_values_workspace_bytes(5, 5, 10) >= 256


def test_minplus_and_variant_entry_points_reject_bad_arguments_before_device_work():
    P = ctypes.c_void_p
    fake = P(256)
    lib = binding.lib
    for T, m, B, shared in ((0, 3, 4, 1), (2, 0, 4, 1), (2, 5000, 4, 1), (2, 3, 0, 0), (2, 3, 4, 2)):
        assert lib.split_minplus_forward_device(fake, shared, T, m, B, fake, fake, None, None) == \
            binding.SPLIT_EINVAL, (T, m, B, shared)
    assert lib.split_minplus_forward_device(None, 1, 2, 3, 4, fake, fake, None, None) == binding.SPLIT_EINVAL
    assert lib.split_minplus_backtrack_device(fake, None, 2, 3, 4, fake, None) == binding.SPLIT_EINVAL
    for U, T, B, R, u, rho in ((-1, 1, 1, 1, 0, 0), (5000, 1, 1, 1, 0, 0), (3, 0, 1, 1, 0, 0), (3, 1, 1, 0, 0, 0),
                               (3, 1, 1, 65, 0, 0), (3, 1, 1, 2, -1, 0), (3, 1, 1, 2, 0, -1)):
        assert lib.split_ou_transitions_device(U, T, B, R, fake, fake, fake, fake, u, rho, fake, None) == \
            binding.SPLIT_EINVAL, (U, T, B, R, u, rho)
    for U, T, B, R, u, rho in ((-1, 1, 1, 1, 0, 0), (32, 1, 1, 1, 0, 0), (3, 0, 1, 1, 0, 0), (3, 1, 0, 1, 0, 0),
                               (3, 1, 1 << 31, 1, 0, 0), (3, 1, 1, 0, 0, 0), (3, 1, 1, 65, 0, 0), (3, 1, 1, 2, -1, 0),
                               (3, 1, 1, 2, 0, -1)):
        assert lib.split_ou_dp_device(U, T, B, R, fake, fake, fake, fake, u, rho, fake, fake, None, None, None) == \
            binding.SPLIT_EINVAL, (U, T, B, R, u, rho)
    assert lib.split_ou_dp_device(3, 1, 1, 1, fake, fake, fake, fake, 0, 0, None, fake, None, None, None) == \
        binding.SPLIT_EINVAL
    f = lib.split_variant_device
    assert f(fake, 5, fake, 5, fake, 10, 3, 1 << 24, 0, fake, fake, fake, 1 << 20, None) == binding.SPLIT_EINVAL
    assert f(fake, 5, fake, 5, fake, 10, 3, 2, -1, fake, fake, fake, 1 << 20, None) == binding.SPLIT_EINVAL
    assert f(fake, 5, fake, 5, fake, 10, 3, 2, 0, fake, None, fake, 1 << 20, None) == binding.SPLIT_EINVAL
    assert f(fake, 5, fake, 5, fake, 10, 3, 2, 0, fake, fake, fake, 16, None) == binding.SPLIT_EINVAL
    assert binding.variant_workspace_bytes(200, 200, 10 ** 6, 4) > binding.variant_workspace_bytes(200, 200, 10 ** 6, 0)


def test_path_choice_of_the_one_launch_form():
    """split_eval_path (host logic only): one tour, at most 256 recursion
    steps per wave of the 8-wave workgroup, pools of at most 256 customers,
    automatic path choice; anything else takes the general kernels."""
    P = binding.eval_path
    assert P(1, 20, 20, 1000, 30) == binding.PATH_ONE_LAUNCH       # n=20, S=1000
    assert P(1, 128, 200, 1024, 100) == binding.PATH_ONE_LAUNCH    # 2 tiles per wave x 128
    assert P(1, 128, 200, 1025, 100) == binding.PATH_TILES         # 3 tiles per wave
    assert P(1, 256, 256, 512, 100) == binding.PATH_ONE_LAUNCH
    assert P(1, 257, 256, 512, 100) == binding.PATH_TILES
    assert P(1, 20, 256, 1000, 30) == binding.PATH_ONE_LAUNCH
    assert P(1, 20, 257, 1000, 30) == binding.PATH_ORDERED        # large pools: tour-ordered copy
    assert P(2, 20, 100, 1000, 30) == binding.PATH_TILES
    assert P(1, 0, 100, 1000, 30) == binding.PATH_TILES
    assert P(1, 100, 200, 100_000, 100) == binding.PATH_TILES
    for bad in ((0, 20, 100, 1000, 30), (1, 20, 100, 0, 30), (1, 20, 0, 1000, 30)):
        with pytest.raises(binding.SplitError):
            P(*bad)
    try:
        binding.set_schedule(32, 8, 3, 3, waves=0, path=1)
        assert P(1, 20, 20, 1000, 30) == binding.PATH_TILES
        binding.set_schedule(32, 8, 3, 3, waves=0, path=0)
        assert P(1, 20, 20, 1000, 30) == binding.PATH_ONE_LAUNCH
        binding.profile_enable(True)
        assert P(1, 20, 20, 1000, 30) == binding.PATH_TILES
    finally:
        binding.profile_enable(False)
        binding.set_schedule(0)


def test_tuned_entry_with_path_zero_selects_the_one_launch_form(tmp_path):
    """A recorded path 0 (the tuner's record of the one-launch form) keeps
    the automatic choice; a recorded path 1 forces the general kernels."""
    binding.tune_clear()
    key = (0, 4, 4, 4, 4)  # one tour, n~20, N~20, S~1000, Q~30
    try:
        for path, want in ((0, binding.PATH_ONE_LAUNCH), (1, binding.PATH_TILES)):
            f = tmp_path / ("tune%d.txt" % path)
            f.write_text("%d %d %d %d %d 32 8 3 3 0 %d\n" % (key + (path,)))
            binding.tune_load(f)
            assert binding.tune_lookup(1, 20, 20, 1000, 30) == (32, 8, 3, 3, 0, path)
            assert binding.eval_path(1, 20, 20, 1000, 30) == want
            binding.tune_clear()
    finally:
        binding.tune_clear()
