#!/usr/bin/env python
"""Benchmark of the scenario-batched split evaluator on one MI355X.

Headline (one JSON line on stdout): Bellman cells/s of the plain split at
the paper's scale -- one giant tour of n=200 customers, S=10^6 demand
scenarios, Q=150 -- with all inputs resident in HBM before timing starts.
A step is one full evaluation (per-tour constants, the window recursion for
every scenario, exact fallback, per-tour sum and mean).

Also reported on the same line: scenarios/s, the main kernel's roofline
(int32 VALU ops, one per Bellman cell, against the chip's VALU peak), the
CPU oracle's throughput on a bounded sample of the same workload, route
recovery of the same tour (predecessors and cut points of every scenario),
the split variants (soft capacity, fleet bound), the order-up-to inventory
DP on the generic min-plus update, the candidate search under a fixed time
budget (GPU vs CPU oracle as evaluator), the batched form (256 ragged tours in one captured graph vs one launch per
tour) and the served form.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Bellman cells/s & scenarios/s at n=200,S=1e6; batched vs plain; p99 latency"
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz plain 32-bit VALU lane-ops/s
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2602_05179_amd/csrc/split_kernels.hip",
                  "paper_2602_05179_amd/csrc/window_min_asm.inc",
                  "paper_2602_05179_amd/csrc/split_internal.h",
                  "paper_2602_05179_amd/csrc/split_device.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_split_tile_n200_S1e6.txt")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "sq_counters_split_tile_n200_S1e6.md")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha1()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def read_traffic():
    """HBM bytes per launch of the main kernel from the committed rocprofv3
    counter summary, or None if absent or taken on a different kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_hash") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_valu_counters():
    """VALU instructions per launch of the main kernel from the committed
    rocprofv3 SQ-counter summary, or None if absent or taken on a different
    kernel."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    text = open(COUNTERS_FILE).read()
    if "kernel_hash = %s " % kernel_hash() not in text:
        return None
    for line in text.splitlines():
        cols = [c.strip() for c in line.split("|")]
        if len(cols) > 2 and cols[1] == "SQ_INSTS_VALU":
            try:
                return float(cols[2])
            except ValueError:
                return None
    return None


def timed_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def cpu_baseline(inst):
    """The oracle (as it stands) on a bounded sample of the same workload:
    the median of at least five passes over every scenario on all usable
    host threads (more passes while under about 12 s of CPU time), then one
    thread on a prefix."""
    import numpy as np
    import oracle
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    times, cells = [], 0.0
    while len(times) < 5 or (sum(times) * cores < 12.0 and sum(times) < 30.0):
        t0 = time.perf_counter()
        r = oracle.split_eval(inst.tours, inst.lens, inst.dist, inst.demands, inst.Q, nthreads=cores)
        times.append(time.perf_counter() - t0)
        cells = float(r["cells"].sum())
    t_med = float(np.median(times))
    S_one = min(inst.S, 250_000)
    t0 = time.perf_counter()
    r1 = oracle.split_eval(inst.tours, inst.lens, inst.dist, inst.demands[:S_one], inst.Q, nthreads=1)
    t_one = time.perf_counter() - t0
    return {
        "value": cells / t_med,
        "unit": "cells/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "all %d scenarios, median of %d passes on %d threads (%.3f s per pass, %.1f s CPU in all); "
                  "scenarios/s %.4g; 1 thread: first %d scenarios (%.2f s), %.4g cells/s" % (
                      inst.S, len(times), cores, t_med, sum(times) * cores, inst.S / t_med, S_one, t_one,
                      float(r1["cells"].sum()) / t_one),
        "cells_per_scenario_sample": cells / inst.S,
    }


def batched_vs_plain(torch, binding, W, reps):
    """256 ragged tours on 10^4 shared scenarios: one graph vs one launch per tour."""
    inst = W.batched_ragged(4)
    tours, lens, dist, dem = W.as_arrays(inst)
    dev = torch.device("cuda:0")
    t = torch.from_numpy(tours).to(dev)
    l = torch.from_numpy(lens).to(dev)
    d = torch.from_numpy(dist).to(dev)
    q = torch.from_numpy(dem).to(dev)
    T, max_len = inst.num_tours, int(lens.max())
    cells = int(binding.split_count_cells_device(t, l, q, inst.N, inst.Q).sum().item())
    plan = binding.Plan(t, l, d, q, inst.Q, max_len=max_len)
    t_graph = timed_steps(torch, plan.launch, reps, 2)
    ws = torch.empty(binding.workspace_bytes(T, max_len, inst.N, inst.S, inst.Q), dtype=torch.uint8, device=dev)
    out = binding.DeviceOutputs(T, inst.S, dev)
    t_eager = timed_steps(torch, lambda: binding.split_eval_device(t, l, d, q, inst.Q, max_len=max_len, out=out,
                                                                   workspace=ws), reps, 2)
    offs = [0]
    for n in lens:
        offs.append(offs[-1] + int(n))
    singles = []
    for k in range(T):
        n = int(lens[k])
        singles.append((t[offs[k]:offs[k] + n], l[k:k + 1], binding.DeviceOutputs(1, inst.S, dev),
                        torch.empty(binding.workspace_bytes(1, max(n, 1), inst.N, inst.S, inst.Q), dtype=torch.uint8,
                                    device=dev), max(n, 1)))

    def plain():
        for tt, ll, oo, ww, ml in singles:
            binding.split_eval_device(tt, ll, d, q, inst.Q, max_len=ml, out=oo, workspace=ww)

    t_plain_host = timed_steps(torch, plain, max(1, reps // 4), 1)
    # the same 256 one-tour launches captured in one graph, so that the
    # comparison is between device work and not host launch overhead
    t_plain_graph = None
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            plain()
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plain()
        t_plain_graph = timed_steps(torch, g.replay, reps, 2)
    except RuntimeError as e:  # capture refused: keep the host-loop figure only
        log("plain per-tour graph capture failed: %s" % e)
    same = all(torch.equal(singles[k][2].costs[0], plan.out.costs[k]) for k in range(T))
    same = same and all(torch.equal(singles[k][2].sums, plan.out.sums[k:k + 1]) for k in range(T))
    plan.close()
    t_plain = t_plain_graph if t_plain_graph else t_plain_host
    return {
        "workload": inst.name,
        "cells": cells,
        "batched_graph_ms": t_graph * 1e3,
        "batched_graph_cells_per_s": cells / t_graph,
        "batched_frac_valu_peak": cells / t_graph / 1e12 / VALU_PEAK_TOPS,
        "batched_eager_ms": t_eager * 1e3,
        "plain_per_tour_graph_ms": t_plain_graph * 1e3 if t_plain_graph else None,
        "plain_per_tour_host_loop_ms": t_plain_host * 1e3,
        "plain_per_tour_cells_per_s": cells / t_plain,
        "speedup_batched_vs_plain": t_plain / t_graph,
        "speedup_basis": "256 one-tour launches captured in one graph vs one batched graph" if t_plain_graph
                         else "host loop of 256 one-tour launches vs one batched graph",
        "batched_equals_plain": bool(same),
    }


def latency_small(torch, binding, W, reps=400):
    """Config n=20, S=1000, Q=30: latency of one evaluation (launch to
    result on the host), p50/p99 over repeated calls, for the captured graph
    (inputs resident), the same plan launched eagerly (one library call,
    ordinary kernel launches), the eager device form (arguments checked
    and marshalled per call) and the host form (host buffers in and out,
    copies included)."""
    import numpy as np
    inst = W.plain_small(1, S=1000)
    tours, lens, dist, dem = W.as_arrays(inst)
    dev = torch.device("cuda:0")
    t, l, d, q = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (tours, lens, dist, dem))
    n = int(lens.max())
    cells = int(binding.split_count_cells_device(t, l, q, inst.N, inst.Q).sum().item())
    plan = binding.Plan(t, l, d, q, inst.Q, max_len=n)
    ws = torch.empty(binding.workspace_bytes(1, n, inst.N, inst.S, inst.Q), dtype=torch.uint8, device=dev)
    out = binding.DeviceOutputs(1, inst.S, dev)

    def lat(fn):
        for _ in range(20):
            fn()
        torch.cuda.synchronize()
        xs = np.empty(reps)
        for i in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            xs[i] = time.perf_counter() - t0
        us = xs * 1e6
        return {"p50_us": float(np.percentile(us, 50)), "p99_us": float(np.percentile(us, 99)),
                "mean_us": float(us.mean())}

    res = {"workload": inst.name + ", uniform demands U{1..10}, int32 rounded Euclidean costs",
           "cells": cells, "reps": reps}
    res["graph"] = lat(plan.launch)
    res["plan_eager"] = lat(plan.launch_eager)
    res["eager"] = lat(lambda: binding.split_eval_device(t, l, d, q, inst.Q, max_len=n, out=out, workspace=ws))
    res["host_form"] = lat(lambda: binding.split_eval(tours, lens, dist, dem, inst.Q))
    res["graph_cells_per_s"] = cells / (res["graph"]["p50_us"] * 1e-6)
    plan.close()
    return res


def medium_rotating(torch, binding, W, buffers=16, reps=48):
    """Config n=100, S=10^5, Q=100 (20 MB of demands, small enough to sit in
    the 256 MB Infinity Cache): the main kernel timed with HIP events while
    the calls rotate over `buffers` device copies of the demand tensor, so
    every call reads its demands from HBM."""
    import numpy as np
    inst = W.plain_medium(2, S=100_000)
    tours, lens, dist, dem = W.as_arrays(inst)
    dev = torch.device("cuda:0")
    t, l, d = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (tours, lens, dist))
    qs = [torch.from_numpy(dem).to(dev) for _ in range(buffers)]
    n, S = int(lens.max()), inst.S
    cells = int(binding.split_count_cells_device(t, l, qs[0], inst.N, inst.Q).sum().item())
    ws = torch.empty(binding.workspace_bytes(1, n, inst.N, S, inst.Q), dtype=torch.uint8, device=dev)
    out = binding.DeviceOutputs(1, S, dev)
    ref = None
    for k in range(buffers):
        binding.split_eval_device(t, l, d, qs[k], inst.Q, max_len=n, out=out, workspace=ws)
        c = out.costs.clone()
        ref = c if ref is None else ref
        assert torch.equal(c, ref), "rotating buffers disagree"
    torch.cuda.synchronize()
    binding.profile_read()
    binding.profile_enable(True)
    t0 = time.perf_counter()
    for i in range(reps):
        binding.split_eval_device(t, l, d, qs[i % buffers], inst.Q, max_len=n, out=out, workspace=ws)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    kms, launches = binding.profile_read()
    binding.profile_enable(False)
    kernel_s = kms / 1e3 / max(launches, 1)
    alg_bytes = dem.nbytes + S * 4
    t_valu = cells / (VALU_PEAK_TOPS * 1e12)
    t_hbm = alg_bytes / (HBM_PEAK_GBS * 1e9)
    return {
        "workload": inst.name + ", demands round(Normal(mu,0.3mu))>=1, mu~U{1..20}; %d rotating demand buffers "
                                "(%.0f MB)" % (buffers, buffers * dem.nbytes / 1e6),
        "cells": cells,
        "kernel_ms": kernel_s * 1e3,
        "call_ms": wall * 1e3,
        "cells_per_s": cells / kernel_s,
        "scenarios_per_s": S / kernel_s,
        "roofline": {"bound": "alu" if t_valu >= t_hbm else "hbm",
                     "achieved_tops": cells / kernel_s / 1e12, "achieved_gbs": alg_bytes / kernel_s / 1e9,
                     "frac": max(t_valu, t_hbm) / kernel_s, "algorithmic_bytes": alg_bytes,
                     "t_valu_us": t_valu * 1e6, "t_hbm_us": t_hbm * 1e6},
    }


def route_recovery(torch, binding, t, d, q, inst, cells, eval_costs, steps, warmup):
    """Route recovery of the headline tour over the same S scenarios: the
    smallest minimising predecessor of every position and the route cut
    points of every scenario, inputs resident in HBM."""
    dev = q.device
    n, S = int(t.numel()), inst.S
    out = binding.RouteOutputs(n, S, dev)
    ws = torch.empty(binding.routes_workspace_bytes(n, inst.N, S), dtype=torch.uint8, device=dev)

    def step():
        binding.split_routes_device(t, d, q, inst.Q, out=out, workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    binding.profile_read()
    binding.profile_enable(True)
    sec = timed_steps(torch, step, steps, 0)
    kms, launches = binding.profile_read()
    binding.profile_enable(False)
    kernel_s = kms / 1e3 / max(launches, 1)
    routes_mean = float(out.nroutes.double().mean().item())
    # demands read once; pred for every position; cuts up to nroutes; costs and counts
    alg_bytes = q.numel() * 2 + n * S * 2 + routes_mean * S * 2 + S * 8
    return {
        "workload": "route recovery of the same tour: n=%d, S=%d, Q=%d" % (n, S, inst.Q),
        "ms_per_call": sec * 1e3,
        "cells_per_s": cells / sec,
        "scenarios_per_s": S / sec,
        "kernel": "routes_key_kernel + routes_wide_kernel (one of them returns at once)",
        "kernel_ms": kernel_s * 1e3,
        "kernel_cells_per_s": cells / kernel_s,
        "frac_valu_peak": cells / kernel_s / 1e12 / VALU_PEAK_TOPS,
        "algorithmic_bytes": alg_bytes,
        "achieved_gbs": alg_bytes / kernel_s / 1e9,
        "hbm_frac": alg_bytes / kernel_s / 1e9 / HBM_PEAK_GBS,
        "mean_routes": routes_mean,
        "kernel_vs_eval_kernel": None,
        "costs_equal_eval": bool(torch.equal(out.costs, eval_costs)),
    }


def split_variants(torch, binding, t, d, q, inst, cells, steps, warmup):
    """The split variants on the headline tour and scenarios: soft capacity
    (overload penalty beta per unit) and a fleet bound K (at most K routes).

    Algorithmic work per pass (the roofline's unit, one int32 op each): the
    hard split's Bellman cells; soft capacity adds two ops per position (a
    predecessor that leaves the hard window joins one running minimum once,
    and that minimum is combined with the window's).  A fleet bound of K
    runs K passes over the same windows.  Bytes: demands read once, costs
    written once."""
    dev = q.device
    n, S = int(t.numel()), inst.S
    out = binding.VariantOutputs(S, dev)
    res = {}
    alg_bytes = q.numel() * 2 + S * 4
    for beta, K in ((10, 0), (-1, 25), (10, 25)):
        ws = torch.empty(binding.variant_workspace_bytes(n, inst.N, S, K), dtype=torch.uint8, device=dev)

        def step():
            binding.split_variant_device(t, d, q, inst.Q, beta=beta, K=K, out=out, workspace=ws)

        sec = timed_steps(torch, step, max(1, steps // 4), max(1, warmup // 2))
        status = int(out.status.item())
        key = "beta%d_K%d" % (beta, K)
        per_pass = cells + (2 * n * S if beta >= 0 else 0)
        ops = (K or 1) * per_pass
        t_valu = ops / (VALU_PEAK_TOPS * 1e12)
        t_hbm = alg_bytes / (HBM_PEAK_GBS * 1e9)
        res[key] = {"ms_per_call": sec * 1e3, "scenarios_per_s": S / sec, "status": status,
                    "algorithmic_ops": ops, "ops_per_s": ops / sec,
                    "roofline": {"bound": "alu" if t_valu >= t_hbm else "hbm", "unit": "TOP/s",
                                 "achieved": ops / sec / 1e12, "peak": VALU_PEAK_TOPS,
                                 "frac": max(t_valu, t_hbm) / sec, "basis": "whole call"}}
        del ws
    res["workload"] = "split variants of the same tour: n=%d, S=%d, Q=%d (beta: penalty per unit of " \
                      "overload, -1 = hard capacity; K: fleet bound, 0 = unlimited)" % (n, S, inst.Q)
    return res


def inventory_minplus(torch, binding, W, steps, warmup):
    """The order-up-to inventory DP: the fused kernel (route-option minimum,
    predecessor minimum and recorded minimisers in one launch, no
    transition matrices), then for comparison the two-pass form (transition
    generator writing A, generic min-plus forward reading it), and the
    backtracking.  Algorithmic bytes: demands and route options read once,
    J_0 read, J_T and the minimisers written."""
    import numpy as np
    inst = W.inventory_ou()
    dev = torch.device("cuda:0")
    T, B = inst.demand.shape
    R = inst.opt_cost.shape[2]
    m = inst.U + 1
    dem, cost, cap, h = (torch.from_numpy(np.ascontiguousarray(a)).to(dev)
                         for a in (inst.demand, inst.opt_cost, inst.opt_cap, inst.h))
    J0 = torch.full((B, m), int(binding.MINPLUS_INF), dtype=torch.int32, device=dev)
    J0[torch.arange(B, device=dev), torch.from_numpy(inst.I0.astype(np.int64)).to(dev)] = 0
    res = {}
    fJT = torch.empty((B, m), dtype=torch.int32, device=dev)
    farg = torch.empty((T, B, m), dtype=torch.int32, device=dev)

    def fused():
        binding.ou_dp(inst.U, dem, cost, cap, h, inst.u, inst.rho, J0, out=(fJT, farg))

    t_fused_call = timed_steps(torch, fused, steps, warmup)
    # device time of the launch: a captured graph of `reps` calls, HIP events
    reps = 20
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fused()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fused()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    t_fused = e0.elapsed_time(e1) / 1e3 / reps
    res["fused"] = (fJT, farg)
    A = binding.ou_transitions(inst.U, dem, cost, cap, h, inst.u, inst.rho)
    t_gen = timed_steps(torch, lambda: binding.ou_transitions(inst.U, dem, cost, cap, h, inst.u, inst.rho, out=A),
                        steps, warmup)

    def fwd():
        res["out"] = binding.minplus_forward(A, J0, shared=False)

    t_fwd = timed_steps(torch, fwd, steps, warmup)
    JT, arg = res["out"]
    fJT, farg = res["fused"]
    same = bool(torch.equal(JT, fJT) and torch.equal(arg, farg))
    t_bt = timed_steps(torch, lambda: binding.minplus_backtrack(fJT, farg), steps, warmup)
    alg_bytes = T * B * 4 + 2 * T * B * R * 4 + 2 * B * m * 4 + T * B * m * 4
    a_bytes = T * B * m * m * 4
    del A
    return {
        "workload": inst.name,
        "problems": B,
        "states": m,
        "days": T,
        "fused_ms": t_fused * 1e3,
        "fused_call_ms": t_fused_call * 1e3,
        "fused_algorithmic_bytes": alg_bytes,
        "roofline": {"bound": "hbm", "unit": "GB/s", "achieved": alg_bytes / t_fused / 1e9, "peak": HBM_PEAK_GBS,
                     "frac": alg_bytes / t_fused / 1e9 / HBM_PEAK_GBS,
                     "basis": "device time per launch: HIP events around a captured graph of 20 launches"},
        "fused_problem_days_per_s": T * B / t_fused,
        "fused_equals_two_pass": same,
        "two_pass_generator_ms": t_gen * 1e3,
        "two_pass_forward_ms": t_fwd * 1e3,
        "two_pass_matrix_bytes": a_bytes,
        "speedup_fused_vs_two_pass": (t_gen + t_fwd) / t_fused,
        "backtrack_ms": t_bt * 1e3,
        "mean_terminal_cost": float(fJT.double().min(dim=1).values.mean().item()),
    }


def search_budget(torch, binding, W, budget_s, seed=12):
    """First-stage candidate search under a fixed wall-clock budget (the
    shape of the paper's fixed-time-budget comparison): the same genetic
    algorithm and seed with the GPU evaluator and with the CPU oracle
    (all usable host threads) as evaluator, on one instance with 10^4
    scenarios."""
    import numpy as np
    import oracle
    inst = W.plain_normal(seed, 100, 10_000, 100)
    tours, lens, dist, dem = W.as_arrays(inst)
    dev = torch.device("cuda:0")
    d, q = torch.from_numpy(dist).to(dev), torch.from_numpy(dem).to(dev)
    kw = dict(population=64, offspring=256, time_budget_s=budget_s, mutation=0.3, seed=seed)
    gpu = binding.search(d, q, inst.Q, **kw)
    cores = max(1, min(16, len(os.sched_getaffinity(0))))

    def ev(t):
        return oracle.split_eval(t.ravel(), np.full(t.shape[0], t.shape[1], np.int32), dist, dem, inst.Q,
                                 nthreads=cores)["sums"]

    cpu = binding.search(dist, dem, inst.Q, evaluator=ev, **kw)
    S = inst.S

    def summary(r):
        tr = r["trace"]
        return {"candidates": r["candidates"], "generations": len(tr) - 1, "best_mean": r["best_sum"] / S,
                "candidates_per_s": r["candidates"] / max(tr[-1, 0], 1e-9),
                "first_mean": tr[0, 2] / S}

    return {"workload": "GA over giant tours, n=100, S=10^4, Q=100, population 64, 256 candidates per "
                        "generation, %.0f s budget each, seed %d" % (budget_s, seed),
            "gpu": summary(gpu), "cpu_oracle": dict(summary(cpu), cores=cores)}


def served(torch, binding, W, num_requests, pool_size, budget_gb, seed=5):
    """Served stream: single-tour requests (a fresh giant tour of a resident
    instance, Q uniform over {80,150,300}) over a pool of distinct resident
    instances (n ~ U{50..1000} customers, S ~ 10^U(3,5) scenarios,
    Normal(mu,0.3mu) demands), continuous batching at tile granularity
    under an HBM budget small enough that admission queues.  Saturation
    (every request queued at once; the median of three passes after a
    warm-up pass), then Poisson arrivals at 0.5, 0.8 and 0.95 of the
    saturated rate; latency from submission to the result."""
    import threading

    import numpy as np
    dev = torch.device("cuda:0")
    pool = [req.inst for req in W.served_stream(seed=seed, num_requests=pool_size)]
    rng = np.random.default_rng(seed + 1)
    picks = rng.integers(0, len(pool), size=num_requests)
    qs = rng.choice([80, 150, 300], size=num_requests)
    tours = [rng.permutation(pool[k].N).astype(np.int32) + 1 for k in picks]
    # exact Bellman cells of every request (device counter, before timing)
    cells = np.zeros(num_requests, np.int64)
    by_inst = {}
    for i, k in enumerate(picks):
        by_inst.setdefault(int(k), []).append(i)
    for k, idx in by_inst.items():
        q = torch.from_numpy(np.ascontiguousarray(pool[k].demands)).to(dev)
        for Qv in (80, 150, 300):
            sel = [i for i in idx if qs[i] == Qv]
            if not sel:
                continue
            t = torch.from_numpy(np.concatenate([tours[i] for i in sel])).to(dev)
            l = torch.from_numpy(np.array([tours[i].size for i in sel], np.int32)).to(dev)
            cells[sel] = binding.split_count_cells_device(t, l, q, pool[k].N, int(Qv)).cpu().numpy()
        del q
    torch.cuda.synchronize()
    resident = sum(inst.demands.nbytes for inst in pool)
    srv = binding.Server(int(budget_gb * (1 << 30)), max_len=1024)
    ids = [srv.add_instance(inst.dist, inst.demands) for inst in pool]

    def run(rate):
        """rate None: every request queued at once (saturation)."""
        gaps = rng.exponential(1.0 / rate, size=num_requests) if rate else np.zeros(num_requests)
        arrivals = np.cumsum(gaps)
        rids = [None] * num_requests
        lat = np.zeros(num_requests)
        ready = threading.Semaphore(0)

        def collect():
            for i in range(num_requests):
                ready.acquire()
                lat[i] = srv.wait(rids[i])["latency_s"]

        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for i in range(num_requests):
            if rate:
                delay = arrivals[i] - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
            rids[i] = srv.submit(ids[picks[i]], tours[i], int(qs[i]))
            ready.release()
        th.join()
        wall = time.perf_counter() - t0
        ms = lat * 1e3
        return dict(requests=num_requests, wall_s=wall, req_per_s=num_requests / wall,
                    cells_per_s=float(cells.sum()) / wall, p50_ms=float(np.percentile(ms, 50)),
                    p99_ms=float(np.percentile(ms, 99)), mean_ms=float(ms.mean()))

    log("served: %d resident instances, %.0f MB of demands, %.3g cells per request" % (
        len(pool), resident / 1e6, float(cells.mean())))
    run(None)  # warm-up pass (drain kernels, caches, host threads)
    # three saturated passes; the one with the median rate is reported (a
    # single pass varies by several percent from run to run), all three
    # rates beside it
    passes = sorted((run(None) for _ in range(3)), key=lambda r: r["cells_per_s"])
    sat = dict(passes[1])
    sat["basis"] = "median of 3 saturated passes"
    sat["cells_per_s_passes"] = [p["cells_per_s"] for p in passes]
    log("served saturated: %.0f requests/s, %.3g cells/s (passes %s), p50 %.2f ms, p99 %.2f ms" % (
        sat["req_per_s"], sat["cells_per_s"], ", ".join("%.3g" % p["cells_per_s"] for p in passes),
        sat["p50_ms"], sat["p99_ms"]))
    out = {"workload": "%d requests over %d resident instances: n~U{50..1000}, S~10^U(3,5), "
                       "Q in {80,150,300}, Normal(mu,0.3mu) demands, a fresh tour per request"
                       % (num_requests, len(pool)),
           "budget_gb": budget_gb, "resident_demand_bytes": resident,
           "cells_per_request_mean": float(cells.mean()), "saturated": sat}
    for frac in (0.5, 0.8, 0.95):
        out["load_%g" % frac] = run(frac * sat["req_per_s"])
        log("served at %.2f of saturation: p50 %.2f ms, p99 %.2f ms" % (
            frac, out["load_%g" % frac]["p50_ms"], out["load_%g" % frac]["p99_ms"]))
    st = srv.stats()
    out["capacity_bytes"] = st["capacity"]
    out["peak_bytes"] = st["peak_bytes"]
    out["drain_launches"] = st["drains"]
    out["blocked_rounds"] = st["blocked_rounds"]
    srv.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--scenarios", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the n=20 latency and n=100 sections")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-routes", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-minplus", action="store_true")
    ap.add_argument("--search-budget", type=float, default=5.0,
                    help="seconds per evaluator for the candidate-search comparison (0: skip)")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=10_000)
    ap.add_argument("--served-pool", type=int, default=32)
    ap.add_argument("--budget-gb", type=float, default=8.0)
    ap.add_argument("--calibration-copy", action="store_true",
                    help="also run a plain device copy of the demand tensor (HBM counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the evaluator runs on one GPU; --gpus %d is not supported (use --gpus 1)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_05179_amd import binding
    from paper_2602_05179_amd import workloads as W

    dev = torch.device("cuda:0")
    log("generating n=200 S=%d Q=150 (seed %d)" % (args.scenarios, args.seed))
    inst = W.plain_paper_scale(args.seed, S=args.scenarios)
    tours, lens, dist, dem = W.as_arrays(inst)
    t = torch.from_numpy(tours).to(dev)
    l = torch.from_numpy(lens).to(dev)
    d = torch.from_numpy(dist).to(dev)
    q = torch.from_numpy(dem).to(dev)
    T, N, S, n = inst.num_tours, inst.N, inst.S, int(lens.max())
    ws = torch.empty(binding.workspace_bytes(T, n, N, S, inst.Q), dtype=torch.uint8, device=dev)
    out = binding.DeviceOutputs(T, S, dev)
    cells = int(binding.split_count_cells_device(t, l, q, N, inst.Q).sum().item())
    torch.cuda.synchronize()
    log("inputs resident (%.1f MB demands); %d Bellman cells per step" % (dem.nbytes / 1e6, cells))

    def eager_step():
        binding.split_eval_device(t, l, d, q, inst.Q, max_len=n, out=out, workspace=ws)

    # main-kernel duration: HIP events around each launch, eager launches
    for _ in range(args.warmup):
        eager_step()
    torch.cuda.synchronize()
    binding.profile_read()
    binding.profile_enable(True)
    sec_eager = timed_steps(torch, eager_step, args.steps, 0)
    kms, launches = binding.profile_read()
    binding.profile_enable(False)
    kernel_s = kms / 1e3 / max(launches, 1)

    # the step: one replay of the captured evaluation graph
    plan = binding.Plan(t, l, d, q, inst.Q, max_len=n)
    sec = timed_steps(torch, plan.launch, args.steps, args.warmup)
    same = torch.equal(plan.out.costs, out.costs) and torch.equal(plan.out.sums, out.sums)
    plan.close()
    log("timed %d steps: %.3f ms/step (graph), %.3f ms/step (eager), main kernel %.3f ms" % (
        args.steps, sec * 1e3, sec_eager * 1e3, kernel_s * 1e3))

    if args.calibration_copy:
        for _ in range(3):
            q.clone()
        torch.cuda.synchronize()
        log("calibration copies: 3 x %d bytes read + written" % dem.nbytes)

    alg_bytes = dem.nbytes + S * 4
    achieved = cells / kernel_s / 1e12
    traffic = read_traffic()
    valu_insts = read_valu_counters()
    measured_peak = binding.probe_valu_peak() / 1e12
    log("measured int32 VALU peak %.2f T lane-ops/s (spec %.2f)" % (measured_peak, VALU_PEAK_TOPS))
    result = {
        "metric": METRIC,
        "value": cells / sec,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "plain split, 1 giant tour n=200, S=%d scenarios, Q=150, demands "
                               "round(Normal(mu,0.3mu))>=1 int16 scenario-major, int32 rounded Euclidean costs" % S,
                   "n": n, "S": S, "Q": inst.Q, "seed": args.seed, "cells_per_step": cells},
        "scenarios_per_s": S / sec,
        "eager_ms_per_step": sec_eager * 1e3,
        "graph_equals_eager": bool(same),
        "roofline": {
            "bound": "alu",
            "kernel": "split_tile_kernel",
            "achieved": achieved,
            "peak": VALU_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_TOPS,
            "traffic": traffic,
            "algorithmic_bytes": alg_bytes,
            "achieved_gbs": alg_bytes / kernel_s / 1e9,
            "hbm_frac": alg_bytes / kernel_s / 1e9 / HBM_PEAK_GBS,
            "kernel_ms": kernel_s * 1e3,
            "kernel_hash": kernel_hash(),
            "measured_peak": measured_peak,
            "frac_of_measured_peak": achieved / measured_peak,
            "valu_insts_per_launch": valu_insts,
            "valu_issue_frac": (valu_insts * 64 / kernel_s / 1e12 / VALU_PEAK_TOPS
                                if valu_insts else None),
            "traffic_source": ("committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary %s, taken at this kernel_hash"
                               % os.path.relpath(TRAFFIC_FILE, ROOT)) if traffic is not None else None,
            "valu_insts_source": ("committed rocprofv3 SQ_INSTS_VALU summary %s, taken at this kernel_hash"
                                  % os.path.relpath(COUNTERS_FILE, ROOT)) if valu_insts is not None else None,
            "kernel_ms_source": "HIP events around each main-kernel launch on its stream, in this run",
        },
    }
    if not args.no_small:
        log("latency at n=20, S=1000, Q=30")
        result["latency_n20_S1e3"] = latency_small(torch, binding, W)
        log("n=100, S=10^5, Q=100 over rotating demand buffers")
        result["medium_n100_S1e5"] = medium_rotating(torch, binding, W)
    if not args.no_routes:
        log("route recovery (n=%d, S=%d)" % (n, S))
        rr = route_recovery(torch, binding, t, d, q, inst, cells, out.costs[0], args.steps, args.warmup)
        rr["kernel_vs_eval_kernel"] = rr["kernel_ms"] / (kernel_s * 1e3)
        result["routes"] = rr
    if not args.no_variants:
        log("split variants (soft capacity, fleet bound)")
        result["variants"] = split_variants(torch, binding, t, d, q, inst, cells, args.steps, args.warmup)
    if not args.no_minplus:
        log("inventory DP on the min-plus update")
        result["inventory_minplus"] = inventory_minplus(torch, binding, W, max(2, args.steps // 4), 2)
    if args.search_budget > 0:
        log("candidate search, %.0f s budget per evaluator" % args.search_budget)
        result["search"] = search_budget(torch, binding, W, args.search_budget)
    if not args.no_batched:
        log("batched vs plain (256 ragged tours, S=10^4)")
        result["batched"] = batched_vs_plain(torch, binding, W, reps=20)
    if not args.no_served:
        log("served stream (%d requests)" % args.served_requests)
        result["served"] = served(torch, binding, W, args.served_requests, args.served_pool, args.budget_gb)
    if not args.no_cpu_baseline:
        log("CPU oracle baseline on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(inst)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
