// split_tune.cpp -- schedule autotuner.
//
// A schedule fixes how the main kernel runs: register-ring length, head and
// tail structure of the window minimum, tours per workgroup sharing a staged
// tile, and fused vs ordered path, and for one short tour the one-launch
// form (recorded as path 0, the automatic choice that takes it).  Every candidate gives the same results
// by construction (anything the fast path cannot take goes to the exact
// fallback); the tuner still parity-gates each one against the reference
// schedule on the device (bit-exact costs and sums) before timing counts.
// The fastest schedule is recorded for the call's shape bucket; later calls
// in that bucket use it unless split_set_schedule overrides.  The table can
// be saved to and loaded from a small text file.

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <stdio.h>
#include <vector>

#include "split_eval.h"
#include "split_internal.h"
#include "split_small.h"

namespace splitk {

namespace {

std::mutex g_tune_mu;
std::map<TuneKey, Schedule> g_table;

int bucket_log2(int64_t v)
{
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

} // namespace

bool TuneKey::operator<(const TuneKey &o) const
{
    if (tours != o.tours)
        return tours < o.tours;
    if (len != o.len)
        return len < o.len;
    if (pool != o.pool)
        return pool < o.pool;
    if (scen != o.scen)
        return scen < o.scen;
    return cap < o.cap;
}

TuneKey tune_key(int32_t T, int32_t max_len, int32_t N, int64_t S, int32_t Q)
{
    TuneKey k;
    k.tours = T <= 1 ? 0 : T < 8 ? 1 : T < 64 ? 2 : 3;
    k.len = bucket_log2(max_len > 0 ? max_len : 1);
    k.pool = bucket_log2(N);
    k.scen = bucket_log2(S) / 2;
    k.cap = bucket_log2(Q > 0 ? Q : 1);
    return k;
}

bool tuned_schedule(const TuneKey &k, Schedule *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_table.find(k);
    if (it == g_table.end())
        return false;
    *out = it->second;
    return true;
}

} // namespace splitk

extern "C" {

int split_tune_device(const int32_t *d_tours, const int32_t *d_lens, int32_t num_tours,
                      int32_t max_len, const int32_t *d_dist, int32_t N,
                      const int16_t *d_demands, int64_t S, int32_t Q, int32_t reps,
                      split_stream_t stream, double *best_ms)
{
    using namespace splitk;
    clear_error();
    if (num_tours < 1 || N < 1 || S < 1 || Q < 0 || max_len < 0 || max_len > kMaxLen ||
        reps < 1)
        return set_error(SPLIT_EINVAL, "bad tuning arguments");
    if (!d_tours || !d_lens || !d_dist || !d_demands)
        return set_error(SPLIT_EINVAL, "null pointer argument");
    if (reinterpret_cast<uintptr_t>(d_demands) % 16)
        return set_error(SPLIT_EINVAL, "demands must be 16-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);

    // candidates: every compiled window variant x path x tours per workgroup
    Schedule triples[64];
    const int nt = compiled_schedules(triples, 64);
    std::vector<Schedule> cand;
    const bool can_order = ordered_path_possible(N, max_len);
    for (int i = 0; i < nt; ++i) {
        for (int path = 1; path <= 2; ++path) {
            if (path == 2 && !can_order)
                continue;
            if (path == 1) {
                for (int w = 1; w <= 8; w *= 2) {
                    if (w > 1 && w > num_tours)
                        break;
                    Schedule s = triples[i];
                    s.waves = w;
                    s.path = 1;
                    cand.push_back(s);
                }
            } else {
                Schedule s = triples[i];
                s.path = 2;
                cand.push_back(s);
            }
        }
    }
    // the one-launch form (path 0) for every variant, where the shape allows it
    for (int i = 0; i < nt; ++i) {
        Schedule s = triples[i];
        s.waves = 0;
        s.path = 0;
        if (small_path_fits(num_tours, max_len, N, S, s, false))
            cand.push_back(s);
    }
    // reference: the automatic schedule, placed first
    Schedule ref = default_schedule(N, S, Q);
    ref.path = use_ordered_path(num_tours, N, max_len) ? 2 : 1;
    cand.insert(cand.begin(), ref);

    const size_t ws_bytes = workspace_bytes(num_tours, max_len, N, S, can_order);
    const size_t out_bytes = (size_t)num_tours * (size_t)S * 4;
    void *ws = nullptr, *costs_ref = nullptr, *costs = nullptr, *small = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SPLIT_OK;
    double best = 1e30;
    Schedule best_s = ref;
    std::vector<long long> hsum_ref(num_tours), hsum(num_tours);
    int64_t mismatch = 0;
    if (hipMalloc(&ws, ws_bytes) != hipSuccess || hipMalloc(&costs_ref, out_bytes) != hipSuccess ||
        hipMalloc(&costs, out_bytes) != hipSuccess ||
        hipMalloc(&small, (size_t)num_tours * 16 * 2 + 64) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = set_error(SPLIT_ENOMEM, "tuning buffers");
        goto done;
    }
    {
        int64_t *sums_ref = static_cast<int64_t *>(small);
        double *means_ref = reinterpret_cast<double *>(sums_ref + num_tours);
        int64_t *sums = reinterpret_cast<int64_t *>(means_ref + num_tours);
        double *means = reinterpret_cast<double *>(sums + num_tours);
        int64_t *d_mis = reinterpret_cast<int64_t *>(means + num_tours);
        for (size_t c = 0; c < cand.size(); ++c) {
            const Schedule &s = cand[c];
            const bool ordered = s.path == 2;
            const Workspace w = carve_workspace(ws, num_tours, max_len, N, S, ordered);
            int32_t *out = static_cast<int32_t *>(c == 0 ? costs_ref : costs);
            int64_t *so = c == 0 ? sums_ref : sums;
            double *mo = c == 0 ? means_ref : means;
            auto launch = [&]() {
                if (s.path == 0)
                    return launch_small(d_tours, d_lens, max_len, d_dist, N, d_demands, S, Q, out,
                                        so, mo, w, st, s);
                return launch_eval(d_tours, d_lens, num_tours, max_len, d_dist, N, d_demands, S,
                                   Q, out, so, mo, w, st, s);
            };
            hipError_t e = hipSuccess;
            for (int r = 0; r < 2 && e == hipSuccess; ++r) // warm-up
                e = launch();
            if (e == hipSuccess)
                e = hipEventRecord(e0, st);
            for (int r = 0; r < reps && e == hipSuccess; ++r)
                e = launch();
            if (e == hipSuccess)
                e = hipEventRecord(e1, st);
            if (e == hipSuccess && c > 0)
                e = launch_count_mismatch(static_cast<int32_t *>(costs_ref), out,
                                          (int64_t)num_tours * S, d_mis, st);
            if (e == hipSuccess)
                e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                rc = set_error(SPLIT_EDEVICE, "tuning launch: %s", hipGetErrorString(e));
                goto done;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double per = ms / reps;
            if (c == 0) {
                (void)hipMemcpy(hsum_ref.data(), sums_ref, (size_t)num_tours * 8,
                                hipMemcpyDeviceToHost);
            } else {
                (void)hipMemcpy(hsum.data(), sums, (size_t)num_tours * 8, hipMemcpyDeviceToHost);
                (void)hipMemcpy(&mismatch, d_mis, 8, hipMemcpyDeviceToHost);
                if (mismatch != 0 || hsum != hsum_ref) {
                    rc = set_error(SPLIT_EDEVICE,
                                   "schedule ring=%d first=%d group=%d every=%d waves=%d path=%d "
                                   "differs from the reference in %lld costs",
                                   s.ring, s.first, s.group, s.every, s.waves, s.path,
                                   (long long)mismatch);
                    goto done;
                }
            }
            if (per < best) {
                best = per;
                best_s = s;
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_table[tune_key(num_tours, max_len, N, S, Q)] = best_s;
    }
    if (best_ms)
        *best_ms = best;
done:
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (ws)
        (void)hipFree(ws);
    if (costs_ref)
        (void)hipFree(costs_ref);
    if (costs)
        (void)hipFree(costs);
    if (small)
        (void)hipFree(small);
    return rc;
}

int split_tune_lookup(int32_t num_tours, int32_t max_len, int32_t N, int64_t S, int32_t Q,
                      int32_t sched[6])
{
    splitk::clear_error();
    if (!sched)
        return splitk::set_error(SPLIT_EINVAL, "null pointer argument");
    splitk::Schedule s;
    if (!splitk::tuned_schedule(splitk::tune_key(num_tours, max_len, N, S, Q), &s))
        return SPLIT_EAGAIN;
    sched[0] = s.ring;
    sched[1] = s.first;
    sched[2] = s.group;
    sched[3] = s.every;
    sched[4] = s.waves;
    sched[5] = s.path;
    return SPLIT_OK;
}

int split_tune_save(const char *path)
{
    splitk::clear_error();
    FILE *f = path ? fopen(path, "w") : nullptr;
    if (!f)
        return splitk::set_error(SPLIT_EINVAL, "cannot open %s", path ? path : "(null)");
    std::lock_guard<std::mutex> lk(splitk::g_tune_mu);
    fprintf(f, "# tours len pool scen cap -> ring first group every waves path\n");
    for (const auto &kv : splitk::g_table)
        fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d\n", kv.first.tours, kv.first.len,
                kv.first.pool, kv.first.scen, kv.first.cap, kv.second.ring, kv.second.first,
                kv.second.group, kv.second.every, kv.second.waves, kv.second.path);
    fclose(f);
    return SPLIT_OK;
}

int split_tune_load(const char *path)
{
    splitk::clear_error();
    FILE *f = path ? fopen(path, "r") : nullptr;
    if (!f)
        return splitk::set_error(SPLIT_EINVAL, "cannot open %s", path ? path : "(null)");
    char line[256];
    int loaded = 0;
    std::lock_guard<std::mutex> lk(splitk::g_tune_mu);
    while (fgets(line, sizeof(line), f)) {
        if (line[0] == '#')
            continue;
        splitk::TuneKey k;
        splitk::Schedule s;
        if (sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d", &k.tours, &k.len, &k.pool, &k.scen,
                   &k.cap, &s.ring, &s.first, &s.group, &s.every, &s.waves, &s.path) == 11 &&
            splitk::schedule_supported(s) && s.path >= 0 && s.path <= 2 && s.waves >= 0 &&
            s.waves <= 8) {
            splitk::g_table[k] = s;
            ++loaded;
        }
    }
    fclose(f);
    return loaded > 0 ? SPLIT_OK : splitk::set_error(SPLIT_EINVAL, "no entries in %s", path);
}

int split_tune_clear(void)
{
    splitk::clear_error();
    std::lock_guard<std::mutex> lk(splitk::g_tune_mu);
    splitk::g_table.clear();
    return SPLIT_OK;
}

} // extern "C"
