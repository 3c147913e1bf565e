// split_api.cpp -- host side of the C ABI declared in include/split_eval.h.
//
// Argument checking, device buffer management for the synchronous host
// form, the device form, and plans (HIP-graph capture of the batched form).
// All compute runs in the kernels of split_kernels.hip.

#include <hip/hip_runtime.h>

#include <mutex>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <vector>

#include "split_check.h"
#include "split_eval.h"
#include "split_internal.h"
#include "split_values.h"
#include "split_minplus.h"
#include "split_small.h"
#include "split_variant.h"

namespace {

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    splitk::vset_error(code, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory)
        return fail(SPLIT_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(SPLIT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                                                                      \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return hip_fail(e_, what);                                                           \
    } while (0)

using splitk::check_scalars;
using splitk::check_tours_host;

// Device buffers of the synchronous host form, grown on demand.
struct HostCtx {
    std::mutex mu;
    int device = -1;
    hipStream_t stream = nullptr;
    struct Buf {
        void *p = nullptr;
        size_t cap = 0;
    };
    Buf tours, lens, dist, demands, costs, sums, means, ws;
    Buf in, out;        // packed inputs / outputs of a small call (one copy each way)
    Buf pin;            // pinned host staging of a small call (hipHostMalloc)
    ~HostCtx() = default; // buffers live until process exit
};

// Calls whose inputs plus outputs fit in this many bytes are staged through
// one pinned host buffer: one host-to-device copy of every input, one
// device-to-host copy of every output, instead of one pageable copy per
// array (each a separate staged transfer).
constexpr size_t kPackedMax = 8u << 20;

HostCtx g_ctx;

splitk::Schedule g_override = {0, 0, 0, 0, 0}; // ring 0 = automatic

// Event pairs around main-kernel launches while profiling is enabled.
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<splitk::LaunchEvents> pending, spare;
};

Profiler g_prof;

// Returns events to bracket the next launch (or nullptr when disabled).
hipError_t profile_events(splitk::LaunchEvents *out, bool *use)
{
    std::lock_guard<std::mutex> lock(g_prof.mu);
    *use = g_prof.on;
    if (!g_prof.on)
        return hipSuccess;
    splitk::LaunchEvents ev;
    if (!g_prof.spare.empty()) {
        ev = g_prof.spare.back();
        g_prof.spare.pop_back();
    } else {
        hipError_t e = hipEventCreate(&ev.before);
        if (e == hipSuccess)
            e = hipEventCreate(&ev.after);
        if (e != hipSuccess)
            return e;
    }
    g_prof.pending.push_back(ev);
    *out = ev;
    return hipSuccess;
}

bool profiling()
{
    std::lock_guard<std::mutex> lock(g_prof.mu);
    return g_prof.on;
}

hipError_t ensure(HostCtx::Buf &b, size_t bytes)
{
    if (bytes == 0)
        bytes = 256;
    if (b.cap >= bytes)
        return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess)
            return e;
        b.p = nullptr;
        b.cap = 0;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess)
        b.cap = bytes;
    return e;
}

hipError_t ensure_pinned(HostCtx::Buf &b, size_t bytes)
{
    if (b.cap >= bytes)
        return hipSuccess;
    if (b.p) {
        hipError_t e = hipHostFree(b.p);
        if (e != hipSuccess)
            return e;
        b.p = nullptr;
        b.cap = 0;
    }
    hipError_t e = hipHostMalloc(&b.p, bytes, hipHostMallocDefault);
    if (e == hipSuccess)
        b.cap = bytes;
    return e;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

} // namespace

namespace splitk {

// Schedule for a call: an explicit override, else the tuned entry for the
// shape bucket, else the built-in default; `ordered` tells which path runs.
Schedule choose_schedule(int32_t T, int32_t max_len, int32_t N, int64_t S, int32_t Q,
                         bool *ordered)
{
    Schedule s;
    if (g_override.ring)
        s = g_override;
    else if (!tuned_schedule(tune_key(T, max_len, N, S, Q), &s))
        s = default_schedule(N, S, Q);
    bool ord = s.path ? s.path == 2 : use_ordered_path(T, N, max_len);
    if (!ordered_path_possible(N, max_len))
        ord = false;
    *ordered = ord;
    return s;
}

// One evaluation: the one-launch form for one short tour when it fits and
// profiling is off (its events bracket the general tile kernel), else the
// general launches.
static hipError_t run_eval(const int32_t *tours, const int32_t *lens, int32_t T, int32_t max_len,
                           const int32_t *dist, int32_t N, const int16_t *demands, int64_t S,
                           int32_t Q, int32_t *costs, int64_t *sums, double *means,
                           const Workspace &ws, hipStream_t stream, const Schedule &sched,
                           bool ordered, const LaunchEvents *ev)
{
    if (!profiling() && small_path_fits(T, max_len, N, S, sched, ordered))
        return launch_small(tours, lens, max_len, dist, N, demands, S, Q, costs, sums, means, ws,
                            stream, sched);
    return launch_eval(tours, lens, T, max_len, dist, N, demands, S, Q, costs, sums, means, ws,
                       stream, sched, ev);
}

} // namespace splitk

extern "C" {

int split_set_schedule(int32_t ring, int32_t first, int32_t group, int32_t every, int32_t waves,
                       int32_t path)
{
    splitk::clear_error();
    if (ring == 0) {
        g_override = splitk::Schedule{0, 0, 0, 0, 0, 0};
        return SPLIT_OK;
    }
    const splitk::Schedule s{ring, first, group, every, waves, path};
    if (path < 0 || path > 2)
        return fail(SPLIT_EINVAL, "path must be 0, 1 or 2 (got %d)", path);
    if (waves != 0 && waves != 1 && waves != 2 && waves != 4 && waves != 8)
        return fail(SPLIT_EINVAL, "waves must be 0, 1, 2, 4 or 8 (got %d)", waves);
    if (!splitk::schedule_supported(s))
        return fail(SPLIT_EINVAL, "unsupported window variant ring=%d first=%d group=%d every=%d",
                    ring, first, group, every);
    g_override = s;
    return SPLIT_OK;
}

int split_list_variants(int32_t *out, int32_t cap)
{
    splitk::clear_error();
    if (cap < 0 || (cap > 0 && !out))
        return fail(SPLIT_EINVAL, "bad output buffer");
    splitk::Schedule v[64];
    const int n = splitk::compiled_schedules(v, 64);
    for (int i = 0; i < n && i < cap && i < 64; ++i) {
        out[4 * i] = v[i].ring;
        out[4 * i + 1] = v[i].first;
        out[4 * i + 2] = v[i].group;
        out[4 * i + 3] = v[i].every;
    }
    return n;
}

size_t split_workspace_bytes(int32_t num_tours, int32_t max_len, int32_t N, int64_t S, int32_t Q)
{
    if (num_tours < 1 || max_len < 0 || S < 1 || N < 1)
        return 0;
    bool ordered = false;
    (void)splitk::choose_schedule(num_tours, max_len, N, S, Q, &ordered);
    return splitk::workspace_bytes(num_tours, max_len, N, S, ordered);
}

int split_eval_path(int32_t num_tours, int32_t max_len, int32_t N, int64_t S, int32_t Q)
{
    splitk::clear_error();
    const int rc = check_scalars(num_tours, N, S, Q, max_len);
    if (rc)
        return rc;
    bool ordered = false;
    const splitk::Schedule sched = splitk::choose_schedule(num_tours, max_len, N, S, Q, &ordered);
    if (!profiling() && splitk::small_path_fits(num_tours, max_len, N, S, sched, ordered))
        return SPLIT_PATH_ONE_LAUNCH;
    return ordered ? SPLIT_PATH_ORDERED : SPLIT_PATH_TILES;
}

int split_eval_device(const int32_t *d_tours, const int32_t *d_lens, int32_t num_tours,
                      int32_t max_len, const int32_t *d_dist, int32_t N,
                      const int16_t *d_demands, int64_t S, int32_t Q, int32_t *d_costs,
                      int64_t *d_sums, double *d_means, void *d_workspace, size_t ws_bytes,
                      split_stream_t stream)
{
    splitk::clear_error();
    int rc = check_scalars(num_tours, N, S, Q, max_len);
    if (rc)
        return rc;
    if (!d_tours || !d_lens || !d_dist || !d_demands || !d_costs || !d_sums || !d_means ||
        !d_workspace)
        return fail(SPLIT_EINVAL, "null pointer argument");
    if (reinterpret_cast<uintptr_t>(d_demands) % 16)
        return fail(SPLIT_EINVAL, "demands must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256)
        return fail(SPLIT_EINVAL, "workspace must be 256-byte aligned");
    bool ordered = false;
    const splitk::Schedule sched = splitk::choose_schedule(num_tours, max_len, N, S, Q, &ordered);
    const size_t need = splitk::workspace_bytes(num_tours, max_len, N, S, ordered);
    if (ws_bytes < need)
        return fail(SPLIT_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    const splitk::Workspace ws =
        splitk::carve_workspace(d_workspace, num_tours, max_len, N, S, ordered);
    splitk::LaunchEvents ev;
    bool use_ev = false;
    HIP_TRY(profile_events(&ev, &use_ev), "profile events");
    HIP_TRY(splitk::run_eval(d_tours, d_lens, num_tours, max_len, d_dist, N, d_demands, S, Q,
                             d_costs, d_sums, d_means, ws, static_cast<hipStream_t>(stream),
                             sched, ordered, use_ev ? &ev : nullptr),
            "launch");
    return SPLIT_OK;
}

size_t split_routes_workspace_bytes(int32_t n, int32_t N, int64_t S)
{
    if (n < 0 || n > splitk::kMaxLen || S < 1 || N < 1)
        return 0;
    return splitk::routes_workspace_bytes(n, N, S);
}

int split_routes_set_variant(int32_t ring, int32_t first, int32_t group, int32_t every)
{
    splitk::clear_error();
    if (ring == 0) {
        splitk::set_route_override(splitk::RouteVariant{0, 0, 0, 0});
        return SPLIT_OK;
    }
    const splitk::RouteVariant v{ring, first, group, every};
    if (!splitk::route_variant_supported(v))
        return fail(SPLIT_EINVAL, "unsupported route variant ring=%d first=%d group=%d every=%d",
                    ring, first, group, every);
    splitk::set_route_override(v);
    return SPLIT_OK;
}

int split_routes_set_path(int32_t path)
{
    splitk::clear_error();
    if (path < 0 || path > 2)
        return fail(SPLIT_EINVAL, "route path must be 0, 1 or 2 (got %d)", path);
    splitk::set_route_path(path);
    return SPLIT_OK;
}

int split_routes_list_variants(int32_t *out, int32_t cap)
{
    splitk::clear_error();
    if (cap < 0 || (cap > 0 && !out))
        return fail(SPLIT_EINVAL, "bad output buffer");
    splitk::RouteVariant v[64];
    const int n = splitk::compiled_route_variants(v, 64);
    for (int i = 0; i < n && i < cap && i < 64; ++i) {
        out[4 * i] = v[i].ring;
        out[4 * i + 1] = v[i].first;
        out[4 * i + 2] = v[i].group;
        out[4 * i + 3] = v[i].every;
    }
    return n;
}

int split_routes_device(const int32_t *d_tour, int32_t n, const int32_t *d_dist, int32_t N,
                        const int16_t *d_demands, int64_t S, int32_t Q, int32_t *d_costs,
                        uint16_t *d_pred, uint16_t *d_cuts, int32_t *d_nroutes,
                        void *d_workspace, size_t ws_bytes, split_stream_t stream)
{
    splitk::clear_error();
    int rc = check_scalars(1, N, S, Q, n);
    if (rc)
        return rc;
    if (!d_dist || !d_demands || !d_costs || !d_nroutes || !d_workspace ||
        (n > 0 && (!d_tour || !d_pred || !d_cuts)))
        return fail(SPLIT_EINVAL, "null pointer argument");
    if (reinterpret_cast<uintptr_t>(d_demands) % 16)
        return fail(SPLIT_EINVAL, "demands must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256)
        return fail(SPLIT_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = splitk::routes_workspace_bytes(n, N, S);
    if (ws_bytes < need)
        return fail(SPLIT_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    const splitk::Workspace ws =
        splitk::carve_workspace(d_workspace, 1, n, N, S, splitk::routes_ordered(n, N));
    splitk::LaunchEvents ev;
    bool use_ev = false;
    HIP_TRY(profile_events(&ev, &use_ev), "profile events");
    HIP_TRY(splitk::launch_routes(d_tour, n, d_dist, N, d_demands, S, Q, d_costs, d_pred, d_cuts,
                                  d_nroutes, ws,
                                  splitk::routes_position_table(d_workspace, n, N, S),
                                  static_cast<hipStream_t>(stream),
                                  splitk::choose_route_variant(Q), use_ev ? &ev : nullptr),
            "launch");
    return SPLIT_OK;
}

size_t split_values_workspace_bytes(int32_t n, int32_t N, int64_t S)
{
    if (n < 0 || n > splitk::kMaxLen || S < 1 || N < 1)
        return 0;
    return splitk::workspace_bytes(1, n, N, S, false);
}

int split_values_device(const int32_t *d_tour, int32_t n, const int32_t *d_dist, int32_t N,
                        const int16_t *d_demands, int64_t S, int32_t Q, int32_t *d_V,
                        int32_t *d_status, void *d_workspace, size_t ws_bytes,
                        split_stream_t stream)
{
    splitk::clear_error();
    int rc = check_scalars(1, N, S, Q, n);
    if (rc)
        return rc;
    if (!d_dist || !d_demands || !d_status || !d_workspace || (n > 0 && (!d_tour || !d_V)))
        return fail(SPLIT_EINVAL, "null pointer argument");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256)
        return fail(SPLIT_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = splitk::workspace_bytes(1, n, N, S, false);
    if (ws_bytes < need)
        return fail(SPLIT_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    const splitk::Workspace ws = splitk::carve_workspace(d_workspace, 1, n, N, S, false);
    HIP_TRY(splitk::launch_values(d_tour, n, d_dist, N, d_demands, S, Q, d_V, d_status, ws,
                                  static_cast<hipStream_t>(stream)),
            "launch");
    return SPLIT_OK;
}

int split_variant_set_path(int32_t path)
{
    splitk::clear_error();
    if (path < 0 || path > 2)
        return fail(SPLIT_EINVAL, "variant path must be 0, 1 or 2 (got %d)", path);
    splitk::set_variant_path(path);
    return SPLIT_OK;
}

size_t split_variant_workspace_bytes(int32_t n, int32_t N, int64_t S, int32_t K)
{
    if (n < 0 || n > splitk::kMaxLen || S < 1 || N < 1 || K < 0)
        return 0;
    return splitk::variant_workspace_bytes(n, N, S, K);
}

int split_variant_device(const int32_t *d_tour, int32_t n, const int32_t *d_dist, int32_t N,
                         const int16_t *d_demands, int64_t S, int32_t Q, int32_t beta, int32_t K,
                         int32_t *d_costs, int32_t *d_status, void *d_workspace, size_t ws_bytes,
                         split_stream_t stream)
{
    splitk::clear_error();
    int rc = check_scalars(1, N, S, Q, n);
    if (rc)
        return rc;
    if (K < 0 || K > splitk::kMaxLen)
        return fail(SPLIT_EINVAL, "K must be in [0, %d] (got %d)", splitk::kMaxLen, K);
    if (beta >= (1 << 24))
        return fail(SPLIT_EINVAL, "beta must be below 2^24 (got %d)", beta);
    if (!d_dist || !d_demands || !d_costs || !d_status || !d_workspace || (n > 0 && !d_tour))
        return fail(SPLIT_EINVAL, "null pointer argument");
    if (reinterpret_cast<uintptr_t>(d_demands) % 16)
        return fail(SPLIT_EINVAL, "demands must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256)
        return fail(SPLIT_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = splitk::variant_workspace_bytes(n, N, S, K);
    if (ws_bytes < need)
        return fail(SPLIT_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    HIP_TRY(splitk::launch_variant(d_tour, n, d_dist, N, d_demands, S, Q, beta, K, d_costs,
                                   d_status, d_workspace, static_cast<hipStream_t>(stream)),
            "launch");
    return SPLIT_OK;
}

int split_minplus_forward_device(const int32_t *d_A, int32_t shared, int32_t T, int32_t m,
                                 int64_t B, const int32_t *d_J0, int32_t *d_JT, int32_t *d_arg,
                                 split_stream_t stream)
{
    splitk::clear_error();
    if (T < 1 || m < 1 || m > splitk::kMinplusMaxStates || B < 1 || B > (int64_t)INT32_MAX)
        return fail(SPLIT_EINVAL, "need T >= 1, 1 <= m <= %d, 1 <= B < 2^31 (got T=%d m=%d B=%lld)",
                    splitk::kMinplusMaxStates, T, m, (long long)B);
    if (shared != 0 && shared != 1)
        return fail(SPLIT_EINVAL, "shared must be 0 or 1 (got %d)", shared);
    if (!d_A || !d_J0 || !d_JT)
        return fail(SPLIT_EINVAL, "null pointer argument");
    HIP_TRY(splitk::launch_minplus_forward(d_A, shared, T, m, B, d_J0, d_JT, d_arg,
                                           static_cast<hipStream_t>(stream)),
            "launch");
    return SPLIT_OK;
}

int split_minplus_backtrack_device(const int32_t *d_JT, const int32_t *d_arg, int32_t T,
                                   int32_t m, int64_t B, int32_t *d_path, split_stream_t stream)
{
    splitk::clear_error();
    if (T < 1 || m < 1 || m > splitk::kMinplusMaxStates || B < 1 || B > (int64_t)INT32_MAX)
        return fail(SPLIT_EINVAL, "need T >= 1, 1 <= m <= %d, 1 <= B < 2^31",
                    splitk::kMinplusMaxStates);
    if (!d_JT || !d_arg || !d_path)
        return fail(SPLIT_EINVAL, "null pointer argument");
    HIP_TRY(splitk::launch_minplus_backtrack(d_JT, d_arg, T, m, B, d_path,
                                             static_cast<hipStream_t>(stream)),
            "launch");
    return SPLIT_OK;
}

int split_ou_transitions_device(int32_t U, int32_t T, int64_t B, int32_t R,
                                const int32_t *d_demand, const int32_t *d_opt_cost,
                                const int32_t *d_opt_cap, const int32_t *d_h, int32_t u,
                                int32_t rho, int32_t *d_A, split_stream_t stream)
{
    splitk::clear_error();
    if (U < 0 || U + 1 > splitk::kMinplusMaxStates || T < 1 || B < 1 || R < 1 || R > 64)
        return fail(SPLIT_EINVAL, "need 0 <= U < %d, T >= 1, B >= 1, 1 <= R <= 64",
                    splitk::kMinplusMaxStates);
    if (u < 0 || rho < 0)
        return fail(SPLIT_EINVAL, "u and rho must be >= 0");
    if (!d_demand || !d_opt_cost || !d_opt_cap || !d_h || !d_A)
        return fail(SPLIT_EINVAL, "null pointer argument");
    HIP_TRY(splitk::launch_ou_transitions(U, T, B, R, d_demand, d_opt_cost, d_opt_cap, d_h, u, rho,
                                          d_A, static_cast<hipStream_t>(stream)),
            "launch");
    return SPLIT_OK;
}

int split_ou_dp_device(int32_t U, int32_t T, int64_t B, int32_t R, const int32_t *d_demand,
                       const int32_t *d_opt_cost, const int32_t *d_opt_cap, const int32_t *d_h,
                       int32_t u, int32_t rho, const int32_t *d_J0, int32_t *d_JT,
                       int32_t *d_arg, int32_t *d_status, split_stream_t stream)
{
    splitk::clear_error();
    if (U < 0 || U + 1 > splitk::kOuMaxStates || T < 1 || B < 1 || B > (int64_t)INT32_MAX ||
        R < 1 || R > 64)
        return fail(SPLIT_EINVAL, "need 0 <= U < %d, T >= 1, 1 <= B < 2^31, 1 <= R <= 64 "
                    "(got U=%d T=%d B=%lld R=%d)", splitk::kOuMaxStates, U, T, (long long)B, R);
    if (u < 0 || rho < 0)
        return fail(SPLIT_EINVAL, "u and rho must be >= 0");
    if (!d_demand || !d_opt_cost || !d_opt_cap || !d_h || !d_J0 || !d_JT)
        return fail(SPLIT_EINVAL, "null pointer argument");
    HIP_TRY(splitk::launch_ou_dp(U, T, B, R, d_demand, d_opt_cost, d_opt_cap, d_h, u, rho, d_J0,
                                 d_JT, d_arg, d_status, static_cast<hipStream_t>(stream)),
            "launch");
    return SPLIT_OK;
}

int split_profile_enable(int32_t on)
{
    splitk::clear_error();
    std::lock_guard<std::mutex> lock(g_prof.mu);
    g_prof.on = on != 0;
    return SPLIT_OK;
}

int split_profile_read(double *kernel_ms, int64_t *launches)
{
    splitk::clear_error();
    if (!kernel_ms || !launches)
        return fail(SPLIT_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lock(g_prof.mu);
    double total = 0.0;
    int64_t count = 0;
    for (const splitk::LaunchEvents &ev : g_prof.pending) {
        HIP_TRY(hipEventSynchronize(ev.after), "event synchronize");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev.before, ev.after), "event elapsed");
        total += ms;
        ++count;
        g_prof.spare.push_back(ev);
    }
    g_prof.pending.clear();
    *kernel_ms = total;
    *launches = count;
    return SPLIT_OK;
}

int split_eval(const int32_t *tours, const int32_t *lens, int32_t num_tours, const int32_t *dist,
               int32_t N, const int16_t *demands, int64_t S, int32_t Q, int32_t *costs,
               int64_t *sums, double *means)
{
    splitk::clear_error();
    if (!tours || !lens || !dist || !demands || !costs)
        return fail(SPLIT_EINVAL, "null pointer argument");
    int rc = check_scalars(num_tours, N, S, Q, 0);
    if (rc)
        return rc;
    int32_t max_len = 0;
    int64_t total = 0;
    rc = check_tours_host(tours, lens, num_tours, dist, N, &max_len, &total);
    if (rc)
        return rc;

    std::lock_guard<std::mutex> lock(g_ctx.mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (g_ctx.stream == nullptr || g_ctx.device != dev) {
        HIP_TRY(hipStreamCreateWithFlags(&g_ctx.stream, hipStreamNonBlocking), "stream");
        g_ctx.device = dev;
    }
    hipStream_t st = g_ctx.stream;
    const size_t n1sq = ((size_t)N + 1) * ((size_t)N + 1);
    bool ordered = false;
    const splitk::Schedule sched = splitk::choose_schedule(num_tours, max_len, N, S, Q, &ordered);
    const size_t ws_bytes = splitk::workspace_bytes(num_tours, max_len, N, S, ordered);
    HIP_TRY(ensure(g_ctx.ws, ws_bytes), "alloc workspace");
    const splitk::Workspace ws =
        splitk::carve_workspace(g_ctx.ws.p, num_tours, max_len, N, S, ordered);

    // small calls: inputs packed at 256-byte offsets {tours, lens, dist,
    // demands}, outputs {sums, means, costs}, each side one copy
    const size_t b_tours = (size_t)total * 4, b_lens = (size_t)num_tours * 4,
                 b_dist = n1sq * 4, b_dem = (size_t)S * N * 2, b_costs = (size_t)num_tours * S * 4,
                 b_sm = (size_t)num_tours * 8;
    const size_t i_lens = align256(b_tours), i_dist = i_lens + align256(b_lens),
                 i_dem = i_dist + align256(b_dist), in_bytes = i_dem + b_dem;
    const size_t o_means = align256(b_sm), o_costs = o_means + align256(b_sm),
                 out_bytes = o_costs + b_costs;
    if (in_bytes + out_bytes <= kPackedMax) {
        HIP_TRY(ensure(g_ctx.in, in_bytes), "alloc inputs");
        HIP_TRY(ensure(g_ctx.out, out_bytes), "alloc outputs");
        HIP_TRY(ensure_pinned(g_ctx.pin, in_bytes > out_bytes ? in_bytes : out_bytes),
                "alloc pinned staging");
        char *h = static_cast<char *>(g_ctx.pin.p);
        char *din = static_cast<char *>(g_ctx.in.p);
        char *dout = static_cast<char *>(g_ctx.out.p);
        if (b_tours)
            memcpy(h, tours, b_tours);
        memcpy(h + i_lens, lens, b_lens);
        memcpy(h + i_dist, dist, b_dist);
        memcpy(h + i_dem, demands, b_dem);
        HIP_TRY(hipMemcpyAsync(din, h, in_bytes, hipMemcpyHostToDevice, st), "copy inputs");
        HIP_TRY(splitk::run_eval(reinterpret_cast<int32_t *>(din),
                                 reinterpret_cast<int32_t *>(din + i_lens), num_tours, max_len,
                                 reinterpret_cast<int32_t *>(din + i_dist), N,
                                 reinterpret_cast<int16_t *>(din + i_dem), S, Q,
                                 reinterpret_cast<int32_t *>(dout + o_costs),
                                 reinterpret_cast<int64_t *>(dout),
                                 reinterpret_cast<double *>(dout + o_means), ws, st, sched, ordered,
                                 nullptr),
                "launch");
        // the staging buffer is reused for the outputs: the copy above has
        // completed by the time this one (same stream) starts
        HIP_TRY(hipMemcpyAsync(h, dout, out_bytes, hipMemcpyDeviceToHost, st), "copy outputs");
        HIP_TRY(hipStreamSynchronize(st), "synchronize");
        const int64_t *hs = reinterpret_cast<const int64_t *>(h);
        for (int32_t t = 0; t < num_tours; ++t)
            if (hs[t] == SPLIT_SUM_INVALID)
                return fail(SPLIT_EINVAL, "tour %d: invalid input found on the device "
                                          "(negative demand)", t);
        memcpy(costs, h + o_costs, b_costs);
        if (sums)
            memcpy(sums, h, b_sm);
        if (means)
            memcpy(means, h + o_means, b_sm);
        return SPLIT_OK;
    }

    HIP_TRY(ensure(g_ctx.tours, (size_t)total * 4), "alloc tours");
    HIP_TRY(ensure(g_ctx.lens, (size_t)num_tours * 4), "alloc lens");
    HIP_TRY(ensure(g_ctx.dist, n1sq * 4), "alloc dist");
    HIP_TRY(ensure(g_ctx.demands, (size_t)S * N * 2), "alloc demands");
    HIP_TRY(ensure(g_ctx.costs, (size_t)num_tours * S * 4), "alloc costs");
    HIP_TRY(ensure(g_ctx.sums, (size_t)num_tours * 8), "alloc sums");
    HIP_TRY(ensure(g_ctx.means, (size_t)num_tours * 8), "alloc means");

    if (total)
        HIP_TRY(hipMemcpyAsync(g_ctx.tours.p, tours, (size_t)total * 4, hipMemcpyHostToDevice, st),
                "copy tours");
    HIP_TRY(hipMemcpyAsync(g_ctx.lens.p, lens, (size_t)num_tours * 4, hipMemcpyHostToDevice, st),
            "copy lens");
    HIP_TRY(hipMemcpyAsync(g_ctx.dist.p, dist, n1sq * 4, hipMemcpyHostToDevice, st), "copy dist");
    HIP_TRY(hipMemcpyAsync(g_ctx.demands.p, demands, (size_t)S * N * 2, hipMemcpyHostToDevice, st),
            "copy demands");
    HIP_TRY(splitk::run_eval(static_cast<int32_t *>(g_ctx.tours.p),
                             static_cast<int32_t *>(g_ctx.lens.p), num_tours, max_len,
                             static_cast<int32_t *>(g_ctx.dist.p), N,
                             static_cast<int16_t *>(g_ctx.demands.p), S, Q,
                             static_cast<int32_t *>(g_ctx.costs.p),
                             static_cast<int64_t *>(g_ctx.sums.p),
                             static_cast<double *>(g_ctx.means.p), ws, st, sched, ordered,
                             nullptr),
            "launch");
    std::vector<int64_t> hs(num_tours);
    std::vector<double> hm(num_tours);
    HIP_TRY(hipMemcpyAsync(hs.data(), g_ctx.sums.p, (size_t)num_tours * 8, hipMemcpyDeviceToHost,
                           st),
            "copy sums");
    HIP_TRY(hipMemcpyAsync(hm.data(), g_ctx.means.p, (size_t)num_tours * 8,
                           hipMemcpyDeviceToHost, st),
            "copy means");
    HIP_TRY(hipStreamSynchronize(st), "synchronize");
    for (int32_t t = 0; t < num_tours; ++t)
        if (hs[t] == SPLIT_SUM_INVALID)
            return fail(SPLIT_EINVAL, "tour %d: invalid input found on the device "
                                      "(negative demand)", t);
    HIP_TRY(hipMemcpy(costs, g_ctx.costs.p, (size_t)num_tours * S * 4, hipMemcpyDeviceToHost),
            "copy costs");
    if (sums)
        memcpy(sums, hs.data(), (size_t)num_tours * 8);
    if (means)
        memcpy(means, hm.data(), (size_t)num_tours * 8);
    return SPLIT_OK;
}

int split_count_cells_device(const int32_t *d_tours, const int32_t *d_lens, int32_t num_tours,
                             int32_t N, const int16_t *d_demands, int64_t S, int32_t Q,
                             int64_t *d_cells, split_stream_t stream)
{
    splitk::clear_error();
    int rc = check_scalars(num_tours, N, S, Q, 0);
    if (rc)
        return rc;
    if (!d_tours || !d_lens || !d_demands || !d_cells)
        return fail(SPLIT_EINVAL, "null pointer argument");
    HIP_TRY(splitk::launch_count_cells(d_tours, d_lens, num_tours, N, d_demands, S, Q, d_cells,
                                       static_cast<hipStream_t>(stream)),
            "launch");
    return SPLIT_OK;
}

// ---------------------------------------------------------------------------
// plans: workspace + captured graph
// ---------------------------------------------------------------------------
struct split_plan {
    void *ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // the captured call, for eager replays (split_plan_launch_eager)
    const int32_t *tours = nullptr, *lens = nullptr, *dist = nullptr;
    const int16_t *demands = nullptr;
    int32_t *costs = nullptr;
    int64_t *sums = nullptr;
    double *means = nullptr;
    int32_t T = 0, max_len = 0, N = 0, Q = 0;
    int64_t S = 0;
    splitk::Schedule sched{};
    bool ordered = false;
    splitk::Workspace wsv{};
};

int split_plan_create(split_plan **plan, const int32_t *d_tours, const int32_t *d_lens,
                      int32_t num_tours, int32_t max_len, const int32_t *d_dist, int32_t N,
                      const int16_t *d_demands, int64_t S, int32_t Q, int32_t *d_costs,
                      int64_t *d_sums, double *d_means, split_stream_t stream)
{
    splitk::clear_error();
    if (!plan)
        return fail(SPLIT_EINVAL, "null plan pointer");
    int rc = check_scalars(num_tours, N, S, Q, max_len);
    if (rc)
        return rc;
    split_plan *p = new split_plan();
    const size_t bytes = split_workspace_bytes(num_tours, max_len, N, S, Q);
    hipError_t e = hipMalloc(&p->ws, bytes);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "plan workspace");
    }
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipFree(p->ws);
        delete p;
        return hip_fail(e, "capture stream");
    }
    (void)stream;
    e = splitk::small_prepare(); // one-time kernel set-up outside the capture
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cap);
        (void)hipFree(p->ws);
        delete p;
        return hip_fail(e, "kernel set-up");
    }
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = split_eval_device(d_tours, d_lens, num_tours, max_len, d_dist, N, d_demands, S, Q,
                               d_costs, d_sums, d_means, p->ws, bytes, cap);
        hipError_t e2 = hipStreamEndCapture(cap, &p->graph);
        if (rc == SPLIT_OK && e2 != hipSuccess)
            rc = hip_fail(e2, "end capture");
    } else {
        rc = hip_fail(e, "begin capture");
    }
    if (rc == SPLIT_OK) {
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess)
            rc = hip_fail(e, "graph instantiate");
    }
    if (rc == SPLIT_OK) {
        // the same call as the captured one: the schedule and workspace
        // layout in force at creation
        p->tours = d_tours;
        p->lens = d_lens;
        p->dist = d_dist;
        p->demands = d_demands;
        p->costs = d_costs;
        p->sums = d_sums;
        p->means = d_means;
        p->T = num_tours;
        p->max_len = max_len;
        p->N = N;
        p->Q = Q;
        p->S = S;
        p->sched = splitk::choose_schedule(num_tours, max_len, N, S, Q, &p->ordered);
        p->wsv = splitk::carve_workspace(p->ws, num_tours, max_len, N, S, p->ordered);
    }
    (void)hipStreamDestroy(cap);
    if (rc != SPLIT_OK) {
        if (p->exec)
            (void)hipGraphExecDestroy(p->exec);
        if (p->graph)
            (void)hipGraphDestroy(p->graph);
        (void)hipFree(p->ws);
        delete p;
        return rc;
    }
    *plan = p;
    return SPLIT_OK;
}

int split_plan_launch(split_plan *plan, split_stream_t stream)
{
    splitk::clear_error();
    if (!plan || !plan->exec)
        return fail(SPLIT_EINVAL, "null plan");
    HIP_TRY(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)), "graph launch");
    return SPLIT_OK;
}

int split_plan_launch_eager(split_plan *plan, split_stream_t stream)
{
    splitk::clear_error();
    if (!plan || !plan->exec)
        return fail(SPLIT_EINVAL, "null plan");
    HIP_TRY(splitk::run_eval(plan->tours, plan->lens, plan->T, plan->max_len, plan->dist, plan->N,
                             plan->demands, plan->S, plan->Q, plan->costs, plan->sums,
                             plan->means, plan->wsv, static_cast<hipStream_t>(stream),
                             plan->sched, plan->ordered, nullptr),
            "launch");
    return SPLIT_OK;
}

int split_plan_destroy(split_plan *plan)
{
    splitk::clear_error();
    if (!plan)
        return SPLIT_OK;
    if (plan->exec)
        (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph)
        (void)hipGraphDestroy(plan->graph);
    if (plan->ws)
        (void)hipFree(plan->ws);
    delete plan;
    return SPLIT_OK;
}

} // extern "C"
