"""Thin ctypes binding of libsplit_eval.so (C ABI in include/split_eval.h).

Argument marshalling only: every step of the evaluation runs in the HIP
kernels of the library.  PyTorch is used for device memory and streams.
Importing this module raises if the shared library has not been built:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build_lib import LIB as LIB_PATH

SPLIT_OK = 0
SPLIT_EINVAL = -1
SPLIT_ENOMEM = -2
SPLIT_EDEVICE = -3
SPLIT_EAGAIN = -4
SPLIT_INF = np.iinfo(np.int32).max
SPLIT_SUM_INVALID = np.iinfo(np.int64).min
SPLIT_NO_PRED = 0xFFFF

EXPORTED = (
    "split_last_error",
    "split_eval_device_noalloc",
    "split_noalloc_scratch_bytes",
    "split_ou_dp_device",
    "split_eval",
    "split_workspace_bytes",
    "split_eval_device",
    "split_eval_path",
    "split_count_cells_device",
    "split_plan_create",
    "split_plan_launch",
    "split_plan_launch_eager",
    "split_plan_destroy",
    "split_set_schedule",
    "split_list_variants",
    "split_probe_valu_peak",
    "split_profile_enable",
    "split_profile_read",
    "split_server_create",
    "split_server_add_instance",
    "split_server_remove_instance",
    "split_server_submit",
    "split_server_submit_copy",
    "split_debug_fail_allocations",
    "split_server_poll",
    "split_server_wait",
    "split_server_stats",
    "split_server_destroy",
    "split_tune_device",
    "split_tune_lookup",
    "split_tune_save",
    "split_tune_load",
    "split_tune_clear",
    "split_routes_workspace_bytes",
    "split_values_workspace_bytes",
    "split_values_device",
    "split_routes_device",
    "split_routes_set_variant",
    "split_routes_list_variants",
    "split_routes_set_path",
    "split_variant_workspace_bytes",
    "split_variant_set_path",
    "split_variant_device",
    "split_minplus_forward_device",
    "split_minplus_backtrack_device",
    "split_ou_transitions_device",
    "split_search_run",
)


class SearchParams(ctypes.Structure):
    _fields_ = [("population", ctypes.c_int32), ("offspring", ctypes.c_int32), ("generations", ctypes.c_int32),
                ("time_budget_s", ctypes.c_double), ("mutation", ctypes.c_double), ("seed", ctypes.c_uint64)]


SEARCH_EVAL_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                  ctypes.c_int32, ctypes.POINTER(ctypes.c_int64))


class SplitError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("split library error %d: %s" % (code, msg))
        self.code = code


class ServerStats(ctypes.Structure):
    """split_server_stats_t"""
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("pending", ctypes.c_int64),
                ("running", ctypes.c_int64), ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
                ("capacity", ctypes.c_size_t), ("drains", ctypes.c_int64), ("instances", ctypes.c_int64),
                ("deferred_bytes", ctypes.c_size_t), ("blocked_rounds", ctypes.c_int64)]


def _load():
    # PyTorch-ROCm ships its own HIP runtime under the same soname; loading it
    # first makes this library bind to that one copy instead of a second one.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsplit_eval.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.split_last_error.restype = ctypes.c_char_p
    lib.split_last_error.argtypes = []
    lib.split_eval.restype = ctypes.c_int
    lib.split_eval.argtypes = [P, P, i32, P, i32, P, i64, i32, P, P, P]
    lib.split_workspace_bytes.restype = sz
    lib.split_workspace_bytes.argtypes = [i32, i32, i32, i64, i32]
    lib.split_eval_device.restype = ctypes.c_int
    lib.split_eval_device.argtypes = [P, P, i32, i32, P, i32, P, i64, i32, P, P, P, P, sz, P]
    lib.split_count_cells_device.restype = ctypes.c_int
    lib.split_count_cells_device.argtypes = [P, P, i32, i32, P, i64, i32, P, P]
    lib.split_plan_create.restype = ctypes.c_int
    lib.split_plan_create.argtypes = [ctypes.POINTER(P), P, P, i32, i32, P, i32, P, i64, i32, P, P, P, P]
    lib.split_plan_launch.restype = ctypes.c_int
    lib.split_plan_launch.argtypes = [P, P]
    lib.split_plan_launch_eager.restype = ctypes.c_int
    lib.split_plan_launch_eager.argtypes = [P, P]
    lib.split_plan_destroy.restype = ctypes.c_int
    lib.split_plan_destroy.argtypes = [P]
    lib.split_set_schedule.restype = ctypes.c_int
    lib.split_set_schedule.argtypes = [i32, i32, i32, i32, i32, i32]
    lib.split_probe_valu_peak.restype = ctypes.c_int
    lib.split_probe_valu_peak.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    lib.split_eval_path.restype = ctypes.c_int
    lib.split_eval_path.argtypes = [i32, i32, i32, ctypes.c_int64, i32]
    lib.split_list_variants.restype = ctypes.c_int
    lib.split_list_variants.argtypes = [ctypes.POINTER(i32), i32]
    lib.split_profile_enable.restype = ctypes.c_int
    lib.split_profile_enable.argtypes = [i32]
    lib.split_profile_read.restype = ctypes.c_int
    lib.split_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.split_server_create.restype = ctypes.c_int
    lib.split_server_create.argtypes = [ctypes.POINTER(P), sz, i32]
    lib.split_server_add_instance.restype = ctypes.c_int
    lib.split_server_add_instance.argtypes = [P, P, i32, P, i64, ctypes.POINTER(i64)]
    lib.split_server_remove_instance.restype = ctypes.c_int
    lib.split_server_remove_instance.argtypes = [P, i64]
    lib.split_server_submit.restype = ctypes.c_int
    lib.split_server_submit.argtypes = [P, i64, P, i32, i32, P, ctypes.POINTER(i64)]
    lib.split_server_submit_copy.restype = ctypes.c_int
    lib.split_server_submit_copy.argtypes = [P, P, i32, P, i32, P, i64, i32, P, ctypes.POINTER(i64)]
    lib.split_server_poll.restype = ctypes.c_int
    lib.split_server_poll.argtypes = [P, i64, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
    lib.split_server_wait.restype = ctypes.c_int
    lib.split_server_wait.argtypes = [P, i64]
    lib.split_server_stats.restype = ctypes.c_int
    lib.split_server_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    lib.split_server_destroy.restype = ctypes.c_int
    lib.split_debug_fail_allocations.restype = ctypes.c_int
    lib.split_debug_fail_allocations.argtypes = [i32]
    lib.split_server_destroy.argtypes = [P]
    lib.split_tune_device.restype = ctypes.c_int
    lib.split_tune_device.argtypes = [P, P, i32, i32, P, i32, P, i64, i32, i32, P, ctypes.POINTER(ctypes.c_double)]
    lib.split_tune_lookup.restype = ctypes.c_int
    lib.split_tune_lookup.argtypes = [i32, i32, i32, i64, i32, ctypes.POINTER(i32)]
    lib.split_tune_save.restype = ctypes.c_int
    lib.split_tune_save.argtypes = [ctypes.c_char_p]
    lib.split_tune_load.restype = ctypes.c_int
    lib.split_tune_load.argtypes = [ctypes.c_char_p]
    lib.split_tune_clear.restype = ctypes.c_int
    lib.split_tune_clear.argtypes = []
    lib.split_routes_workspace_bytes.restype = sz
    lib.split_routes_workspace_bytes.argtypes = [i32, i32, i64]
    lib.split_values_workspace_bytes.restype = sz
    lib.split_values_workspace_bytes.argtypes = [i32, i32, i64]
    lib.split_values_device.restype = ctypes.c_int
    lib.split_values_device.argtypes = [P, i32, P, i32, P, i64, i32, P, P, P, sz, P]
    lib.split_routes_device.restype = ctypes.c_int
    lib.split_routes_device.argtypes = [P, i32, P, i32, P, i64, i32, P, P, P, P, P, sz, P]
    lib.split_routes_set_variant.restype = ctypes.c_int
    lib.split_routes_set_variant.argtypes = [i32, i32, i32, i32]
    lib.split_routes_list_variants.restype = ctypes.c_int
    lib.split_routes_set_path.restype = ctypes.c_int
    lib.split_routes_set_path.argtypes = [i32]
    lib.split_variant_set_path.restype = ctypes.c_int
    lib.split_variant_set_path.argtypes = [i32]
    lib.split_variant_workspace_bytes.restype = sz
    lib.split_variant_workspace_bytes.argtypes = [i32, i32, i64, i32]
    lib.split_variant_device.restype = ctypes.c_int
    lib.split_search_run.restype = ctypes.c_int
    lib.split_search_run.argtypes = [P, i32, P, i64, i32, P, ctypes.POINTER(SearchParams), P, P, P,
                                     ctypes.POINTER(i64), ctypes.POINTER(i64), P, i32, ctypes.POINTER(i32), P]
    lib.split_minplus_forward_device.restype = ctypes.c_int
    lib.split_minplus_forward_device.argtypes = [P, i32, i32, i32, i64, P, P, P, P]
    lib.split_minplus_backtrack_device.restype = ctypes.c_int
    lib.split_minplus_backtrack_device.argtypes = [P, P, i32, i32, i64, P, P]
    lib.split_ou_transitions_device.restype = ctypes.c_int
    lib.split_ou_transitions_device.argtypes = [i32, i32, i64, i32, P, P, P, P, i32, i32, P, P]
    lib.split_variant_device.argtypes = [P, i32, P, i32, P, i64, i32, i32, i32, P, P, P, sz, P]
    lib.split_routes_list_variants.argtypes = [ctypes.POINTER(i32), i32]
    lib.split_ou_dp_device.restype = ctypes.c_int
    lib.split_ou_dp_device.argtypes = [i32, i32, i64, i32, P, P, P, P, i32, i32, P, P, P, P, P]
    lib.split_eval_device_noalloc.restype = ctypes.c_int
    lib.split_eval_device_noalloc.argtypes = [P, P, i32, i32, P, i32, P, i64, i32, P, P, P, P]
    lib.split_noalloc_scratch_bytes.restype = sz
    lib.split_noalloc_scratch_bytes.argtypes = []
    return lib


lib = _load()


def last_error() -> str:
    return lib.split_last_error().decode()


def _check(rc: int):
    if rc != SPLIT_OK:
        raise SplitError(rc, last_error())


def list_variants():
    """Compiled window variants as (ring, first, group, every) tuples."""
    n = lib.split_list_variants(None, 0)
    buf = (ctypes.c_int32 * (4 * n))()
    lib.split_list_variants(buf, n)
    return [tuple(int(buf[4 * i + k]) for k in range(4)) for i in range(n)]


SCHEDULES = list_variants()


PATH_AUTO, PATH_FUSED, PATH_ORDERED = 0, 1, 2

PATH_ONE_LAUNCH, PATH_TILES = 0, 1


def eval_path(num_tours: int, max_len: int, N: int, S: int, Q: int) -> int:
    """Kernels an evaluation of this shape runs under the schedule in force:
    PATH_ONE_LAUNCH, PATH_TILES or PATH_ORDERED (the same value as PATH_ORDERED)."""
    rc = lib.split_eval_path(int(num_tours), int(max_len), int(N), int(S), int(Q))
    _check(rc if rc < 0 else 0)
    return rc


def set_schedule(ring: int, first: int = 8, group: int = 0, every: int = 4, waves: int = 0,
                 path: int = 0):
    """Force the main-kernel schedule; ring=0 restores the automatic choice."""
    _check(lib.split_set_schedule(int(ring), int(first), int(group), int(every), int(waves),
                                  int(path)))


def probe_valu_peak(stream=None) -> float:
    """Measured int32 VALU lane-operations per second of the current device."""
    v = ctypes.c_double()
    _check(lib.split_probe_valu_peak(ctypes.byref(v), _stream_handle(stream)))
    return v.value


def profile_enable(on: bool = True):
    """Bracket every main-kernel launch with HIP events (measurement)."""
    _check(lib.split_profile_enable(1 if on else 0))


def profile_read():
    """(summed main-kernel milliseconds, launches) since the last read."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib.split_profile_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------------------
# host form
# ---------------------------------------------------------------------------
def split_eval(tours, lens, dist, demands, Q):
    """Host arrays in, host arrays out (synchronous).

    Returns dict(costs=int32[T, S], sums=int64[T], means=float64[T])."""
    tours = np.ascontiguousarray(tours, np.int32)
    lens = np.ascontiguousarray(lens, np.int32)
    dist = np.ascontiguousarray(dist, np.int32)
    demands = np.ascontiguousarray(demands, np.int16)
    T = int(lens.size)
    N = int(dist.shape[0] - 1)
    S = int(demands.shape[0])
    if demands.ndim != 2 or demands.shape[1] != N or dist.shape != (N + 1, N + 1):
        raise SplitError(SPLIT_EINVAL, "shape mismatch: dist %s demands %s" % (dist.shape, demands.shape))
    if int(lens.sum()) != tours.size:
        raise SplitError(SPLIT_EINVAL, "sum(lens) != len(tours)")
    costs = np.empty((T, S), np.int32)
    sums = np.empty(T, np.int64)
    means = np.empty(T, np.float64)
    _check(lib.split_eval(_np_ptr(tours), _np_ptr(lens), T, _np_ptr(dist), N, _np_ptr(demands), S, int(Q),
                          _np_ptr(costs), _np_ptr(sums), _np_ptr(means)))
    return dict(costs=costs, sums=sums, means=means)


# ---------------------------------------------------------------------------
# device form (torch tensors on the GPU)
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def workspace_bytes(num_tours: int, max_len: int, N: int, S: int, Q: int) -> int:
    return int(lib.split_workspace_bytes(int(num_tours), int(max_len), int(N), int(S), int(Q)))


class DeviceOutputs:
    def __init__(self, T: int, S: int, device):
        torch = _torch()
        self.costs = torch.empty((T, S), dtype=torch.int32, device=device)
        self.sums = torch.empty(T, dtype=torch.int64, device=device)
        self.means = torch.empty(T, dtype=torch.float64, device=device)


def split_eval_device(tours, lens, dist, demands, Q, *, max_len=None, out=None, workspace=None,
                      stream=None):
    """Enqueue an evaluation on device tensors; returns DeviceOutputs.

    tours int32 [sum(lens)], lens int32 [T], dist int32 [N+1, N+1],
    demands int16 [S, N] (16-byte aligned), all on the same GPU."""
    torch = _torch()
    T = int(lens.numel())
    N = int(dist.shape[0] - 1)
    S = int(demands.shape[0])
    for name, t, dt in (("tours", tours, torch.int32), ("lens", lens, torch.int32),
                        ("dist", dist, torch.int32), ("demands", demands, torch.int16)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise SplitError(SPLIT_EINVAL, "%s must be a contiguous %s CUDA tensor" % (name, dt))
    if max_len is None:
        max_len = int(lens.max().item()) if T else 0
    if out is None:
        out = DeviceOutputs(T, S, demands.device)
    need = workspace_bytes(T, max_len, N, S, Q)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=demands.device)
    _check(lib.split_eval_device(_dptr(tours), _dptr(lens), T, int(max_len), _dptr(dist), N, _dptr(demands), S,
                                 int(Q), _dptr(out.costs), _dptr(out.sums), _dptr(out.means), _dptr(workspace),
                                 int(workspace.numel()), _stream_handle(stream)))
    out.workspace = workspace
    return out


def split_eval_device_noalloc(tours, lens, dist, demands, Q, *, max_len=None, out=None, stream=None):
    """split_eval_device with its scratch in the library's fixed device array
    (no workspace argument, no allocation by the library).  Calls that
    overlap on one device share that array and race."""
    T = int(lens.numel())
    N = int(dist.shape[0] - 1)
    S = int(demands.shape[0])
    if max_len is None:
        max_len = int(lens.max().item()) if T else 0
    out = out if out is not None else DeviceOutputs(T, S, demands.device)
    _check(lib.split_eval_device_noalloc(_dptr(tours), _dptr(lens), T, int(max_len), _dptr(dist), N,
                                         _dptr(demands), S, int(Q), _dptr(out.costs), _dptr(out.sums),
                                         _dptr(out.means), _stream_handle(stream)))
    return out


def noalloc_scratch_bytes() -> int:
    """Size of the fixed device array behind split_eval_device_noalloc."""
    return int(lib.split_noalloc_scratch_bytes())


def split_count_cells_device(tours, lens, demands, N, Q, *, stream=None):
    """Number of capacity-admissible relaxations per tour (int64 tensor)."""
    torch = _torch()
    T = int(lens.numel())
    S = int(demands.shape[0])
    cells = torch.empty(T, dtype=torch.int64, device=demands.device)
    _check(lib.split_count_cells_device(_dptr(tours), _dptr(lens), T, int(N), _dptr(demands), S, int(Q),
                                        _dptr(cells), _stream_handle(stream)))
    return cells


# ---------------------------------------------------------------------------
# route recovery (one giant tour, device tensors)
# ---------------------------------------------------------------------------
def list_route_variants():
    """Compiled route-recovery window variants as (ring, first, group, every) tuples."""
    n = lib.split_routes_list_variants(None, 0)
    buf = (ctypes.c_int32 * (4 * n))()
    lib.split_routes_list_variants(buf, n)
    return [tuple(int(buf[4 * i + k]) for k in range(4)) for i in range(n)]


ROUTE_VARIANTS = list_route_variants()


def set_route_variant(ring: int, first: int = 8, group: int = 3, every: int = 3):
    """Force the route-recovery window variant; ring=0 restores the automatic choice."""
    _check(lib.split_routes_set_variant(int(ring), int(first), int(group), int(every)))


ROUTE_PATH_AUTO, ROUTE_PATH_LDS, ROUTE_PATH_ORDERED = 0, 1, 2


def set_route_path(path: int):
    """How route recovery reads the demands: 0 automatic, 1 the tile staged
    in LDS, 2 the tour-ordered copy in the workspace."""
    _check(lib.split_routes_set_path(int(path)))


def routes_workspace_bytes(n: int, N: int, S: int) -> int:
    return int(lib.split_routes_workspace_bytes(int(n), int(N), int(S)))


class RouteOutputs:
    """costs int32 [S]; pred and cuts position-major [n, S] 16-bit words
    (held as int16 tensors, unsigned values: see host()); nroutes int32 [S]."""

    def __init__(self, n: int, S: int, device):
        torch = _torch()
        self.n, self.S = n, S
        self.costs = torch.empty(S, dtype=torch.int32, device=device)
        self.pred = torch.empty((n, S), dtype=torch.int16, device=device)
        self.cuts = torch.empty((n, S), dtype=torch.int16, device=device)
        self.nroutes = torch.empty(S, dtype=torch.int32, device=device)

    def host(self):
        """Copies as numpy: costs, pred uint16 [n, S], cuts uint16 [n, S] (entries
        past nroutes unspecified), nroutes."""
        return dict(costs=self.costs.cpu().numpy(), pred=self.pred.cpu().numpy().view(np.uint16),
                    cuts=self.cuts.cpu().numpy().view(np.uint16), nroutes=self.nroutes.cpu().numpy())


def split_routes_device(tour, dist, demands, Q, *, out=None, workspace=None, stream=None):
    """Enqueue route recovery of one giant tour over every scenario.

    tour int32 [n], dist int32 [N+1, N+1], demands int16 [S, N] (16-byte
    aligned), all on the same GPU.  Returns RouteOutputs."""
    torch = _torch()
    n = int(tour.numel())
    N = int(dist.shape[0] - 1)
    S = int(demands.shape[0])
    for name, t, dt in (("tour", tour, torch.int32), ("dist", dist, torch.int32),
                        ("demands", demands, torch.int16)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise SplitError(SPLIT_EINVAL, "%s must be a contiguous %s CUDA tensor" % (name, dt))
    if out is None:
        out = RouteOutputs(n, S, demands.device)
    elif out.n != n or out.S != S:
        raise SplitError(SPLIT_EINVAL, "outputs sized for n=%d S=%d" % (out.n, out.S))
    need = routes_workspace_bytes(n, N, S)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=demands.device)
    _check(lib.split_routes_device(_dptr(tour), n, _dptr(dist), N, _dptr(demands), S, int(Q),
                                   _dptr(out.costs), _dptr(out.pred), _dptr(out.cuts), _dptr(out.nroutes),
                                   _dptr(workspace), int(workspace.numel()), _stream_handle(stream)))
    out.workspace = workspace
    return out


def values_workspace_bytes(n: int, N: int, S: int) -> int:
    return int(lib.split_values_workspace_bytes(int(n), int(N), int(S)))


def split_values_device(tour, dist, demands, Q, *, V=None, status=None, workspace=None, stream=None):
    """Enqueue the full value table of one giant tour: V int32 [n, S] with
    V[j-1, s] = V_s(j) (SPLIT_INF where infeasible).  Returns (V, status)
    with status an int32 [1] device tensor (1: a negative demand was read)."""
    torch = _torch()
    n = int(tour.numel())
    N = int(dist.shape[0] - 1)
    S = int(demands.shape[0])
    for name, t, dt in (("tour", tour, torch.int32), ("dist", dist, torch.int32),
                        ("demands", demands, torch.int16)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise SplitError(SPLIT_EINVAL, "%s must be a contiguous %s CUDA tensor" % (name, dt))
    if V is None:
        V = torch.empty((n, S), dtype=torch.int32, device=demands.device)
    elif tuple(V.shape) != (n, S) or V.dtype != torch.int32 or not V.is_contiguous():
        raise SplitError(SPLIT_EINVAL, "V must be a contiguous int32 tensor of shape (%d, %d)" % (n, S))
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=demands.device)
    need = values_workspace_bytes(n, N, S)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=demands.device)
    _check(lib.split_values_device(_dptr(tour), n, _dptr(dist), N, _dptr(demands), S, int(Q),
                                   _dptr(V) if n else None, _dptr(status), _dptr(workspace),
                                   int(workspace.numel()), _stream_handle(stream)))
    return V, status


# ---------------------------------------------------------------------------
# split variants: soft capacity (overload penalty) and a fleet bound
# ---------------------------------------------------------------------------
VARIANT_BAD_TOUR, VARIANT_BAD_DEMAND, VARIANT_PENALTY_RANGE = 1, 2, 4


def set_variant_path(path: int):
    """How the split variants read the demands: 0 automatic, 1 the tile
    staged in LDS, 2 the tour-ordered copy in the workspace."""
    _check(lib.split_variant_set_path(int(path)))


def variant_workspace_bytes(n: int, N: int, S: int, K: int) -> int:
    return int(lib.split_variant_workspace_bytes(int(n), int(N), int(S), int(K)))


class VariantOutputs:
    """costs int32 [S]; status int32 [1] (0 = valid)."""

    def __init__(self, S: int, device):
        torch = _torch()
        self.S = S
        self.costs = torch.empty(S, dtype=torch.int32, device=device)
        self.status = torch.empty(1, dtype=torch.int32, device=device)


def split_variant_device(tour, dist, demands, Q, *, beta=-1, K=0, out=None, workspace=None, stream=None):
    """Enqueue the split variant of one giant tour over every scenario:
    overload penalty beta per unit (beta < 0: hard capacity) and at most K
    routes (K = 0: unlimited).  Returns VariantOutputs."""
    torch = _torch()
    n = int(tour.numel())
    N = int(dist.shape[0] - 1)
    S = int(demands.shape[0])
    for name, t, dt in (("tour", tour, torch.int32), ("dist", dist, torch.int32),
                        ("demands", demands, torch.int16)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise SplitError(SPLIT_EINVAL, "%s must be a contiguous %s CUDA tensor" % (name, dt))
    if out is None:
        out = VariantOutputs(S, demands.device)
    need = variant_workspace_bytes(n, N, S, K)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=demands.device)
    _check(lib.split_variant_device(_dptr(tour), n, _dptr(dist), N, _dptr(demands), S, int(Q), int(beta), int(K),
                                    _dptr(out.costs), _dptr(out.status), _dptr(workspace), int(workspace.numel()),
                                    _stream_handle(stream)))
    out.workspace = workspace
    return out


# ---------------------------------------------------------------------------
# min-plus Bellman updates and the order-up-to inventory instance
# ---------------------------------------------------------------------------
MINPLUS_INF = np.iinfo(np.int32).max


def _check_i32(name, t):
    torch = _torch()
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise SplitError(SPLIT_EINVAL, "%s must be a contiguous int32 CUDA tensor" % name)


def minplus_forward(A, J0, *, shared, record_arg=True, stream=None):
    """A: int32 [T, m, m] (shared) or [T, B, m, m]; J0 int32 [B, m].
    Returns (J_T [B, m], arg [T, B, m] or None)."""
    torch = _torch()
    _check_i32("A", A)
    _check_i32("J0", J0)
    B, m = int(J0.shape[0]), int(J0.shape[1])
    T = int(A.shape[0])
    want = (T, m, m) if shared else (T, B, m, m)
    if tuple(A.shape) != want:
        raise SplitError(SPLIT_EINVAL, "A has shape %s, expected %s" % (tuple(A.shape), want))
    JT = torch.empty((B, m), dtype=torch.int32, device=J0.device)
    arg = torch.empty((T, B, m), dtype=torch.int32, device=J0.device) if record_arg else None
    _check(lib.split_minplus_forward_device(_dptr(A), 1 if shared else 0, T, m, B, _dptr(J0), _dptr(JT),
                                            _dptr(arg) if arg is not None else None, _stream_handle(stream)))
    return JT, arg


def ou_dp(U, demand, opt_cost, opt_cap, h, u, rho, J0, *, record_arg=True, status=None, out=None, stream=None):
    """The order-up-to inventory DP in one launch (no transition matrices):
    demand int32 [T, B], opt_cost / opt_cap int32 [T, B, R], h int32 [U+1],
    J0 int32 [B, U+1].  Returns (J_T [B, U+1], arg [T, B, U+1] or None);
    `out`: a (J_T, arg) pair of preallocated tensors to write instead.
    `status`: an int32 device tensor of one element that receives 1 when a
    negative demand, option cost or h entry was read (else 0), or None."""
    torch = _torch()
    for name, t in (("demand", demand), ("opt_cost", opt_cost), ("opt_cap", opt_cap), ("h", h), ("J0", J0)):
        _check_i32(name, t)
    T, B = (int(x) for x in demand.shape)
    R = int(opt_cost.shape[2])
    m = int(U) + 1
    if tuple(opt_cost.shape) != (T, B, R) or tuple(opt_cap.shape) != (T, B, R) or tuple(h.shape) != (m,) \
            or tuple(J0.shape) != (B, m):
        raise SplitError(SPLIT_EINVAL, "shape mismatch: demand %s opt_cost %s opt_cap %s h %s J0 %s" % (
            tuple(demand.shape), tuple(opt_cost.shape), tuple(opt_cap.shape), tuple(h.shape), tuple(J0.shape)))
    if out is not None:
        JT, arg = out
        _check_i32("JT", JT)
        if tuple(JT.shape) != (B, m) or (arg is not None and (tuple(arg.shape) != (T, B, m) or
                                                           not arg.is_contiguous() or arg.dtype != torch.int32)):
            raise SplitError(SPLIT_EINVAL, "out tensors have the wrong shape or type")
    else:
        JT = torch.empty((B, m), dtype=torch.int32, device=J0.device)
        arg = torch.empty((T, B, m), dtype=torch.int32, device=J0.device) if record_arg else None
    _check(lib.split_ou_dp_device(int(U), T, B, R, _dptr(demand), _dptr(opt_cost), _dptr(opt_cap), _dptr(h),
                                  int(u), int(rho), _dptr(J0), _dptr(JT), _dptr(arg) if arg is not None else None,
                                  _dptr(status) if status is not None else None, _stream_handle(stream)))
    return JT, arg


def minplus_backtrack(JT, arg, *, stream=None):
    """State path int32 [T+1, B] from J_T [B, m] and arg [T, B, m]."""
    torch = _torch()
    _check_i32("JT", JT)
    _check_i32("arg", arg)
    T, B, m = (int(x) for x in arg.shape)
    path = torch.empty((T + 1, B), dtype=torch.int32, device=JT.device)
    _check(lib.split_minplus_backtrack_device(_dptr(JT), _dptr(arg), T, m, B, _dptr(path),
                                              _stream_handle(stream)))
    return path


def ou_transitions(U, demand, opt_cost, opt_cap, h, u, rho, *, out=None, stream=None):
    """Transition matrices int32 [T, B, U+1, U+1] of the order-up-to instance.
    demand int32 [T, B]; opt_cost, opt_cap int32 [T, B, R]; h int32 [U+1]."""
    torch = _torch()
    for name, t in (("demand", demand), ("opt_cost", opt_cost), ("opt_cap", opt_cap), ("h", h)):
        _check_i32(name, t)
    T, B = (int(x) for x in demand.shape)
    R = int(opt_cost.shape[2])
    if tuple(opt_cost.shape) != (T, B, R) or tuple(opt_cap.shape) != (T, B, R) or h.numel() != U + 1:
        raise SplitError(SPLIT_EINVAL, "shape mismatch")
    if out is None:
        out = torch.empty((T, B, U + 1, U + 1), dtype=torch.int32, device=demand.device)
    _check(lib.split_ou_transitions_device(int(U), T, B, R, _dptr(demand), _dptr(opt_cost), _dptr(opt_cap),
                                           _dptr(h), int(u), int(rho), _dptr(out), _stream_handle(stream)))
    return out


# ---------------------------------------------------------------------------
# first-stage candidate search (genetic algorithm over giant tours)
# ---------------------------------------------------------------------------
def search(dist, demands, Q, *, population=64, offspring=256, generations=0, time_budget_s=0.0, mutation=0.3,
           seed=1, init_tour=None, evaluator=None, trace_cap=100000, stream=None):
    """Run the search over permutations of 1..N.  dist and demands are
    device tensors (int32 [N+1, N+1], int16 [S, N]) for the GPU evaluator;
    with `evaluator` (a Python callable(tours int32 [count, n] numpy) ->
    int64 [count] sums replacing it) only their shapes are used.  Returns dict(best_tour, best_sum,
    candidates, trace float64 [generations+1, 3] = (seconds, candidates, best sum))."""
    N = int(dist.shape[0] - 1)
    S = int(demands.shape[0])
    params = SearchParams(int(population), int(offspring), int(generations), float(time_budget_s),
                          float(mutation), int(seed))
    best = np.empty(N, np.int32)
    best_sum, cand, tlen = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    trace = np.zeros((max(int(trace_cap), 1), 3), np.float64)
    init = None
    if init_tour is not None:
        init = np.ascontiguousarray(init_tour, np.int32)
    cb = None
    if evaluator is not None:
        def _cb(ctx, tours_p, count, n, sums_p):
            try:
                tours = np.ctypeslib.as_array(tours_p, shape=(count * n,)).reshape(count, n).copy()
                out = np.asarray(evaluator(tours), dtype=np.int64)
                np.ctypeslib.as_array(sums_p, shape=(count,))[:] = out
                return 0
            except Exception:  # reported to the caller as an evaluator error
                return 1
        cb = SEARCH_EVAL_FN(_cb)
    on_gpu = evaluator is None
    _check(lib.split_search_run(_dptr(dist) if on_gpu else None, N, _dptr(demands) if on_gpu else None, S, int(Q),
                                _np_ptr(init) if init is not None else None, ctypes.byref(params),
                                ctypes.cast(cb, ctypes.c_void_p) if cb is not None else None, None,
                                _np_ptr(best), ctypes.byref(best_sum), ctypes.byref(cand), _np_ptr(trace),
                                int(trace_cap), ctypes.byref(tlen), _stream_handle(stream) if on_gpu else None))
    n_tr = min(int(tlen.value), int(trace_cap))
    return dict(best_tour=best, best_sum=int(best_sum.value), candidates=int(cand.value), trace=trace[:n_tr].copy())


def tune_device(tours, lens, dist, demands, Q, *, max_len=None, reps=5, stream=None) -> float:
    """Time every compiled schedule on these device inputs (parity-gated) and
    record the fastest for their shape bucket; returns its ms per evaluation."""
    T = int(lens.numel())
    if max_len is None:
        max_len = int(lens.max().item()) if T else 0
    best = ctypes.c_double()
    _check(lib.split_tune_device(_dptr(tours), _dptr(lens), T, int(max_len), _dptr(dist), int(dist.shape[0] - 1),
                                 _dptr(demands), int(demands.shape[0]), int(Q), int(reps), _stream_handle(stream),
                                 ctypes.byref(best)))
    return best.value


def tune_lookup(num_tours, max_len, N, S, Q):
    """Recorded (ring, first, group, every, waves, path) for the shape, or None."""
    out = (ctypes.c_int32 * 6)()
    rc = lib.split_tune_lookup(int(num_tours), int(max_len), int(N), int(S), int(Q), out)
    if rc == SPLIT_EAGAIN:
        return None
    _check(rc)
    return tuple(int(x) for x in out)


def tune_save(path):
    _check(lib.split_tune_save(str(path).encode()))


def tune_load(path):
    _check(lib.split_tune_load(str(path).encode()))


def tune_clear():
    _check(lib.split_tune_clear())


class Plan:
    """Batched form: workspace + captured HIP graph over fixed device buffers."""

    def __init__(self, tours, lens, dist, demands, Q, max_len, out=None, stream=None):
        T = int(lens.numel())
        N = int(dist.shape[0] - 1)
        S = int(demands.shape[0])
        self.out = out if out is not None else DeviceOutputs(T, S, demands.device)
        self._keep = (tours, lens, dist, demands)
        self._h = ctypes.c_void_p()
        _check(lib.split_plan_create(ctypes.byref(self._h), _dptr(tours), _dptr(lens), T, int(max_len), _dptr(dist),
                                     N, _dptr(demands), S, int(Q), _dptr(self.out.costs), _dptr(self.out.sums),
                                     _dptr(self.out.means), _stream_handle(stream)))

    def launch(self, stream=None):
        _check(lib.split_plan_launch(self._h, _stream_handle(stream)))
        return self.out

    def launch_eager(self, stream=None):
        """The same evaluation as ordinary kernel launches (no graph launch)."""
        _check(lib.split_plan_launch_eager(self._h, _stream_handle(stream)))
        return self.out

    def close(self):
        if self._h:
            lib.split_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Served form (C ABI split_server_*): continuous batching of single-tour
    requests under an HBM budget.  Instances (cost matrix + demand scenarios,
    host arrays) are registered once and stay resident; requests are tours
    evaluated on them, or tours that bring their own instance."""

    def __init__(self, budget_bytes: int = 0, max_len: int = 1024):
        self._h = ctypes.c_void_p()
        _check(lib.split_server_create(ctypes.byref(self._h), int(budget_bytes), int(max_len)))
        self._costs = {}

    def add_instance(self, dist, demands) -> int:
        dist = np.ascontiguousarray(dist, np.int32)
        demands = np.ascontiguousarray(demands, np.int16)
        iid = ctypes.c_int64()
        _check(lib.split_server_add_instance(self._h, _np_ptr(dist), int(dist.shape[0] - 1), _np_ptr(demands),
                                             int(demands.shape[0]), ctypes.byref(iid)))
        return iid.value

    def remove_instance(self, iid: int):
        _check(lib.split_server_remove_instance(self._h, int(iid)))

    def submit(self, iid: int, tour, Q, S: int = 0, *, want_costs=False) -> int:
        """Evaluate `tour` on resident instance `iid` (S = its scenario count,
        needed only with want_costs)."""
        tour = np.ascontiguousarray(tour, np.int32)
        costs = np.empty(int(S), np.int32) if want_costs else None
        rid = ctypes.c_int64()
        _check(lib.split_server_submit(self._h, int(iid), _np_ptr(tour) if tour.size else None, int(tour.size),
                                       int(Q), _np_ptr(costs) if costs is not None else None, ctypes.byref(rid)))
        self._costs[rid.value] = costs
        return rid.value

    def submit_copy(self, tour, dist, demands, Q, *, want_costs=False) -> int:
        tour = np.ascontiguousarray(tour, np.int32)
        dist = np.ascontiguousarray(dist, np.int32)
        demands = np.ascontiguousarray(demands, np.int16)
        costs = np.empty(int(demands.shape[0]), np.int32) if want_costs else None
        rid = ctypes.c_int64()
        _check(lib.split_server_submit_copy(self._h, _np_ptr(tour) if tour.size else None, int(tour.size),
                                            _np_ptr(dist), int(dist.shape[0] - 1), _np_ptr(demands),
                                            int(demands.shape[0]), int(Q),
                                            _np_ptr(costs) if costs is not None else None, ctypes.byref(rid)))
        self._costs[rid.value] = costs
        return rid.value

    def poll(self, rid: int):
        """None while pending or running, else dict(sum, mean, latency_s, costs)."""
        sm, mn, lat = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        rc = lib.split_server_poll(self._h, int(rid), ctypes.byref(sm), ctypes.byref(mn), ctypes.byref(lat))
        if rc == SPLIT_EAGAIN:
            return None
        costs = self._costs.pop(int(rid), None)
        _check(rc)
        return dict(sum=sm.value, mean=mn.value, latency_s=lat.value, costs=costs)

    def wait(self, rid: int):
        _check(lib.split_server_wait(self._h, int(rid)))
        return self.poll(rid)

    def stats(self):
        st = ServerStats()
        _check(lib.split_server_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            lib.split_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._costs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_fail_allocations(count: int):
    """Test hook: the next `count` device reservations of split_server_create
    report out-of-memory."""
    _check(lib.split_debug_fail_allocations(int(count)))
