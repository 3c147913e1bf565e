"""CPU oracle for the scenario-batched split recursion.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
never calls it, and the two share no code.

`split_eval` mirrors the library's contract (per-scenario int32 costs with
INT32_MAX for "no admissible split", exact int64 sums, sum/S means) and is
computed by the plain C loop in split_oracle.c (paper Sec. 2.3 recursion).
`brute` holds an independent enumeration of all cut sets used to pin it.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import brute  # noqa: F401  (re-exported)
from .build import LIB, build_oracle

INF32 = np.iinfo(np.int32).max
INF64 = np.iinfo(np.int64).max

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = build_oracle(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.oracle_split_eval.argtypes = [P, P, i32, P, i32, P, i64, i32, P, P, P, P, ctypes.c_int,
                                          ctypes.c_int]
        lib.oracle_split_eval.restype = ctypes.c_int
        lib.oracle_split_values.argtypes = [P, i32, P, i32, P, i64, ctypes.c_int, P, P]
        lib.oracle_split_values.restype = ctypes.c_int
        lib.oracle_split_routes.argtypes = [P, i32, P, i32, P, i64, i32, P, P, P, P, ctypes.c_int]
        lib.oracle_split_routes.restype = ctypes.c_int
        lib.oracle_split_variant.argtypes = [P, i32, P, i32, P, i64, i32, i32, i32, P, ctypes.c_int]
        lib.oracle_split_variant.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


class OracleError(RuntimeError):
    pass


def split_eval(tours, lens, dist, demands, Q, *, use_break=True, nthreads=1):
    """Evaluate all tours on all scenarios.

    Returns dict(costs=int32[num_tours, S], sums=int64[num_tours],
    means=float64[num_tours], cells=int64[num_tours]).
    """
    lib = _load()
    tours = np.ascontiguousarray(tours, np.int32)
    lens = np.ascontiguousarray(lens, np.int32)
    dist = np.ascontiguousarray(dist, np.int32)
    demands = np.ascontiguousarray(demands, np.int16)
    T = int(lens.size)
    S = int(demands.shape[0])
    N = int(dist.shape[0] - 1)
    if demands.ndim != 2 or demands.shape[1] != N or dist.shape != (N + 1, N + 1):
        raise OracleError("shape mismatch")
    costs = np.empty((T, S), np.int32)
    sums = np.empty(T, np.int64)
    means = np.empty(T, np.float64)
    cells = np.empty(T, np.int64)
    rc = lib.oracle_split_eval(_p(tours), _p(lens), T, _p(dist), N, _p(demands), S, int(Q),
                               _p(costs), _p(sums), _p(means), _p(cells), int(bool(use_break)),
                               int(nthreads))
    if rc != 0:
        raise OracleError("oracle_split_eval returned %d" % rc)
    return dict(costs=costs, sums=sums, means=means, cells=cells)


def split_values(tour, dist, qvis, Q, *, use_break=True):
    """J(0..n) for demands given in visiting order; None where +inf.

    Returns (values list, feasible-cell count)."""
    lib = _load()
    tour = np.ascontiguousarray(tour, np.int32)
    dist = np.ascontiguousarray(dist, np.int32)
    qv = np.ascontiguousarray(qvis, np.int64)
    V = np.empty(tour.size + 1, np.int64)
    cells = np.zeros(1, np.int64)
    rc = lib.oracle_split_values(_p(tour), int(tour.size), _p(dist), int(dist.shape[0] - 1), _p(qv),
                                 int(Q), int(bool(use_break)), _p(V), _p(cells))
    if rc != 0:
        raise OracleError("oracle_split_values returned %d" % rc)
    return [None if v == INF64 else int(v) for v in V], int(cells[0])


NO_PRED = 0xFFFF


def split_routes(tour, dist, demands, Q, *, nthreads=1):
    """Route recovery for one tour over every scenario (smallest minimising
    predecessor, then backtracking from n).

    Returns dict(costs=int32[S], pred=uint16[S, n] (NO_PRED where J(i) is
    +inf), cuts=uint16[S, n] (route ends in increasing order, zeros after),
    nroutes=int32[S])."""
    lib = _load()
    tour = np.ascontiguousarray(tour, np.int32)
    dist = np.ascontiguousarray(dist, np.int32)
    demands = np.ascontiguousarray(demands, np.int16)
    n = int(tour.size)
    S = int(demands.shape[0])
    N = int(dist.shape[0] - 1)
    if demands.ndim != 2 or demands.shape[1] != N or dist.shape != (N + 1, N + 1):
        raise OracleError("shape mismatch")
    costs = np.empty(S, np.int32)
    pred = np.empty((S, n), np.uint16)
    cuts = np.empty((S, n), np.uint16)
    nroutes = np.empty(S, np.int32)
    rc = lib.oracle_split_routes(_p(tour), n, _p(dist), N, _p(demands), S, int(Q), _p(costs),
                                 _p(pred), _p(cuts), _p(nroutes), int(nthreads))
    if rc != 0:
        raise OracleError("oracle_split_routes returned %d" % rc)
    return dict(costs=costs, pred=pred, cuts=cuts, nroutes=nroutes)


def split_variant(tour, dist, demands, Q, *, beta=-1, K=0, nthreads=1):
    """Split variants for one tour over every scenario: soft capacity with
    overload penalty beta per unit (beta < 0: hard capacity) and a fleet of
    at most K routes (K = 0: unlimited).  Returns int64[S] (INF64 where no
    split exists)."""
    lib = _load()
    tour = np.ascontiguousarray(tour, np.int32)
    dist = np.ascontiguousarray(dist, np.int32)
    demands = np.ascontiguousarray(demands, np.int16)
    S = int(demands.shape[0])
    N = int(dist.shape[0] - 1)
    if demands.ndim != 2 or demands.shape[1] != N or dist.shape != (N + 1, N + 1):
        raise OracleError("shape mismatch")
    costs = np.empty(S, np.int64)
    rc = lib.oracle_split_variant(_p(tour), int(tour.size), _p(dist), N, _p(demands), S, int(Q), int(beta),
                                  int(K), _p(costs), int(nthreads))
    if rc != 0:
        raise OracleError("oracle_split_variant returned %d" % rc)
    return costs


__all__ = ["split_eval", "split_values", "split_routes", "split_variant", "brute", "build_oracle",
           "LIB",
           "INF32", "INF64", "NO_PRED", "OracleError"]
