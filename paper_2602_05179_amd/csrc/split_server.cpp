// split_server.cpp -- served form: continuous batching of evaluation
// requests under an HBM budget.
//
// A request is one giant tour with its own cost matrix and demand scenarios
// (device-resident, owned by the caller until the request completes).  The
// server owns one device arena of `budget` bytes; a request is admitted when
// its own device footprint (tour, outputs, workspace) fits in the arena,
// in arrival order, and is then enqueued on one of a few HIP streams, so
// kernels of requests admitted while others are running overlap on the
// device.  A scheduler thread admits, launches and retires requests; a
// retired request's memory returns to the arena at once, which admits the
// next ones.  Results (sum, mean, optionally per-scenario costs) are copied
// to host memory and kept until polled.
//
// The paper's batching loop sizes a batch from free GPU memory and retries
// with a smaller batch on allocation failure (App. B, adaptive batching);
// here the same concern is handled up front by admission against a fixed
// arena, so no device allocation happens while requests run.

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <thread>
#include <unordered_map>
#include <vector>

#include "split_eval.h"
#include "split_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

#define sfail splitk::set_error

// First-fit allocator over one device range (offsets only; 256-byte units).
class Arena {
  public:
    void init(size_t bytes)
    {
        free_.clear();
        free_[0] = bytes;
        cap_ = bytes;
        used_ = 0;
        peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest)
                    free_[start] = rest;
                used_ += bytes;
                peak_ = used_ > peak_ ? used_ : peak_;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t capacity() const { return cap_; }

  private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
};

enum ReqState { PENDING, RUNNING, DONE };

struct Request {
    int64_t id = 0;
    std::vector<int32_t> tour;
    const int32_t *d_dist = nullptr;
    int32_t N = 0;
    const int16_t *d_demands = nullptr;
    int64_t S = 0;
    int32_t Q = 0;
    int32_t *costs_out = nullptr; // host, may be null
    bool ordered = false;
    size_t bytes = 0, off = 0;
    int stream = 0;
    ReqState state = PENDING;
    hipEvent_t done = nullptr;
    Clock::time_point t_submit, t_done;
    // pinned host staging: [0] = n (lens), [1..n] tour; results after
    int32_t *h_in = nullptr;
    int64_t *h_sum = nullptr;
    double *h_mean = nullptr;
    int32_t *h_costs = nullptr; // pinned bounce buffer for costs (if requested)
    int64_t sum = 0;
    double mean = 0.0;
    int error = SPLIT_OK;
};

} // namespace

struct split_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    int device = 0;
    char *arena_base = nullptr;
    Arena arena;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;
    std::deque<Request *> pending;
    std::vector<Request *> running;
    std::unordered_map<int64_t, Request *> all;
    int64_t next_id = 1;
    int64_t submitted = 0, completed = 0;
    int error = SPLIT_OK;
    char error_text[256] = "";

    // device footprint of a request, laid out inside its arena block
    static size_t footprint(const Request &r, size_t *ws_off, size_t *tour_off, size_t *out_off)
    {
        const int32_t n = (int32_t)r.tour.size();
        size_t b = 0;
        *ws_off = b;
        b += (splitk::workspace_bytes(1, n, r.N, r.S, r.ordered) + 255) & ~(size_t)255;
        *tour_off = b;
        b += ((size_t)(n + 1) * 4 + 255) & ~(size_t)255; // lens + tour
        *out_off = b;
        b += ((size_t)r.S * 4 + 16 + 255) & ~(size_t)255; // sums, means, costs
        return b;
    }

    int launch(Request *r)
    {
        size_t ws_off, tour_off, out_off;
        footprint(*r, &ws_off, &tour_off, &out_off);
        char *base = arena_base + r->off;
        int32_t *d_in = reinterpret_cast<int32_t *>(base + tour_off);
        int64_t *d_sum = reinterpret_cast<int64_t *>(base + out_off);
        double *d_mean = reinterpret_cast<double *>(base + out_off + 8);
        int32_t *d_costs = reinterpret_cast<int32_t *>(base + out_off + 16);
        const int32_t n = (int32_t)r->tour.size();
        hipStream_t st = streams[r->stream];
        hipError_t e = hipMemcpyAsync(d_in, r->h_in, (size_t)(n + 1) * 4, hipMemcpyHostToDevice, st);
        if (e != hipSuccess)
            return SPLIT_EDEVICE;
        const splitk::Workspace ws =
            splitk::carve_workspace(base + ws_off, 1, n, r->N, r->S, r->ordered);
        bool ordered = false;
        splitk::Schedule sched = splitk::choose_schedule(1, n, r->N, r->S, r->Q, &ordered);
        if (ordered != r->ordered) // the footprint was sized for r->ordered
            sched = splitk::default_schedule(r->N, r->S, r->Q);
        e = splitk::launch_eval(d_in + 1, d_in, 1, n, r->d_dist, r->N, r->d_demands, r->S, r->Q,
                                d_costs, d_sum, d_mean, ws, st, sched);
        if (e != hipSuccess)
            return SPLIT_EDEVICE;
        e = hipMemcpyAsync(r->h_sum, d_sum, 16, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && r->h_costs)
            e = hipMemcpyAsync(r->h_costs, d_costs, (size_t)r->S * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipEventRecord(r->done, st);
        return e == hipSuccess ? SPLIT_OK : SPLIT_EDEVICE;
    }

    void retire(Request *r)
    {
        r->t_done = Clock::now();
        r->sum = *r->h_sum;
        r->mean = *r->h_mean;
        if (r->error == SPLIT_OK && r->sum == SPLIT_SUM_INVALID)
            r->error = SPLIT_EINVAL;
        if (r->h_costs && r->costs_out)
            memcpy(r->costs_out, r->h_costs, (size_t)r->S * 4);
        arena.release(r->off, r->bytes);
        stream_load[r->stream]--;
        r->state = DONE;
        completed++;
    }

    void loop()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            bool progress = false;
            // admit in arrival order while the arena has room
            while (!pending.empty()) {
                Request *r = pending.front();
                if (!arena.alloc(r->bytes, &r->off))
                    break;
                pending.pop_front();
                int best = 0;
                for (size_t s = 1; s < streams.size(); ++s)
                    if (stream_load[s] < stream_load[best])
                        best = (int)s;
                r->stream = best;
                stream_load[best]++;
                r->state = RUNNING;
                const int rc = launch(r);
                if (rc != SPLIT_OK) {
                    r->error = rc;
                    error = rc;
                    snprintf(error_text, sizeof(error_text), "launch failed for request %lld",
                             (long long)r->id);
                }
                running.push_back(r);
                progress = true;
            }
            // retire finished requests
            for (size_t i = 0; i < running.size();) {
                Request *r = running[i];
                const hipError_t q = r->error ? hipSuccess : hipEventQuery(r->done);
                if (q == hipErrorNotReady) {
                    ++i;
                    continue;
                }
                if (q != hipSuccess) {
                    r->error = SPLIT_EDEVICE;
                    error = SPLIT_EDEVICE;
                }
                retire(r);
                running[i] = running.back();
                running.pop_back();
                progress = true;
            }
            if (progress)
                cv_done.notify_all();
            if (stop && pending.empty() && running.empty())
                break;
            if (!progress) {
                if (running.empty())
                    cv_work.wait(lk, [&] { return stop || !pending.empty(); });
                else
                    cv_work.wait_for(lk, std::chrono::microseconds(20));
            }
        }
    }
};

extern "C" {

int split_server_create(split_server **out, size_t budget_bytes, int32_t num_streams)
{
    splitk::clear_error();
    if (!out || budget_bytes < 4096 || num_streams < 1 || num_streams > 8)
        return sfail(SPLIT_EINVAL, "need budget >= 4096 bytes and 1..8 streams");
    split_server *s = new split_server();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return sfail(SPLIT_EDEVICE, "no device");
    }
    if (hipMalloc(&s->arena_base, budget_bytes) != hipSuccess) {
        delete s;
        return sfail(SPLIT_ENOMEM, "cannot reserve %zu bytes of device memory", budget_bytes);
    }
    s->arena.init(budget_bytes);
    s->streams.resize(num_streams);
    s->stream_load.assign(num_streams, 0);
    for (auto &st : s->streams)
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipFree(s->arena_base);
            delete s;
            return sfail(SPLIT_EDEVICE, "stream creation failed");
        }
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return SPLIT_OK;
}

int split_server_submit(split_server *s, const int32_t *tour, int32_t n, const int32_t *d_dist,
                        int32_t N, const int16_t *d_demands, int64_t S, int32_t Q,
                        int32_t *costs_out, int64_t *id)
{
    splitk::clear_error();
    if (!s || !id || !d_dist || !d_demands || (n > 0 && !tour))
        return sfail(SPLIT_EINVAL, "null argument");
    if (n < 0 || n > splitk::kMaxLen || N < 1 || S < 1 || Q < 0)
        return sfail(SPLIT_EINVAL, "bad sizes n=%d N=%d S=%lld Q=%d", n, N, (long long)S, Q);
    if (reinterpret_cast<uintptr_t>(d_demands) % 16)
        return sfail(SPLIT_EINVAL, "demands must be 16-byte aligned");
    for (int32_t k = 0; k < n; ++k)
        if (tour[k] < 1 || tour[k] > N)
            return sfail(SPLIT_EINVAL, "tour position %d: customer id %d outside [1, %d]", k + 1,
                         tour[k], N);
    Request *r = new Request();
    r->tour.assign(tour, tour + n);
    r->d_dist = d_dist;
    r->N = N;
    r->d_demands = d_demands;
    r->S = S;
    r->Q = Q;
    r->costs_out = costs_out;
    (void)splitk::choose_schedule(1, n, N, S, Q, &r->ordered);
    size_t a, b, c;
    r->bytes = split_server::footprint(*r, &a, &b, &c);
    if (r->bytes > s->arena.capacity()) {
        const size_t need = r->bytes;
        delete r;
        return sfail(SPLIT_ENOMEM, "request needs %zu bytes, the budget is %zu", need,
                     s->arena.capacity());
    }
    // pinned staging: lens + tour, then results
    const size_t pin = (size_t)(n + 1) * 4 + 16 + 16 + (costs_out ? (size_t)S * 4 : 0);
    char *h = nullptr;
    if (hipHostMalloc(reinterpret_cast<void **>(&h), pin, hipHostMallocDefault) != hipSuccess) {
        delete r;
        return sfail(SPLIT_ENOMEM, "pinned staging allocation failed");
    }
    r->h_in = reinterpret_cast<int32_t *>(h);
    r->h_in[0] = n;
    if (n)
        memcpy(r->h_in + 1, tour, (size_t)n * 4);
    char *res = h + (((size_t)(n + 1) * 4 + 15) & ~(size_t)15);
    r->h_sum = reinterpret_cast<int64_t *>(res);
    r->h_mean = reinterpret_cast<double *>(res + 8);
    r->h_costs = costs_out ? reinterpret_cast<int32_t *>(res + 16) : nullptr;
    if (hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(h);
        delete r;
        return sfail(SPLIT_EDEVICE, "event creation failed");
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->id = s->next_id++;
        r->t_submit = Clock::now();
        s->all[r->id] = r;
        s->pending.push_back(r);
        s->submitted++;
        *id = r->id;
    }
    s->cv_work.notify_one();
    return SPLIT_OK;
}

static void free_request(Request *r)
{
    if (r->done)
        (void)hipEventDestroy(r->done);
    if (r->h_in)
        (void)hipHostFree(r->h_in);
    delete r;
}

int split_server_poll(split_server *s, int64_t id, int64_t *sum, double *mean, double *latency_s)
{
    splitk::clear_error();
    if (!s)
        return sfail(SPLIT_EINVAL, "null server");
    Request *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(id);
        if (it == s->all.end())
            return sfail(SPLIT_EINVAL, "unknown request id %lld", (long long)id);
        if (it->second->state != DONE)
            return SPLIT_EAGAIN;
        r = it->second;
        s->all.erase(it);
    }
    const int rc = r->error;
    if (sum)
        *sum = r->sum;
    if (mean)
        *mean = r->mean;
    if (latency_s)
        *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    free_request(r);
    if (rc == SPLIT_EINVAL)
        return sfail(rc, "request %lld: invalid input found on the device", (long long)id);
    return rc == SPLIT_OK ? SPLIT_OK : sfail(rc, "request %lld failed on the device", (long long)id);
}

int split_server_wait(split_server *s, int64_t id)
{
    splitk::clear_error();
    if (!s)
        return sfail(SPLIT_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end())
        return sfail(SPLIT_EINVAL, "unknown request id %lld", (long long)id);
    Request *r = it->second;
    s->cv_done.wait(lk, [&] { return r->state == DONE; });
    return SPLIT_OK;
}

int split_server_stats(split_server *s, int64_t *submitted, int64_t *completed, int64_t *pending,
                       size_t *bytes_in_use, size_t *peak_bytes)
{
    splitk::clear_error();
    if (!s)
        return sfail(SPLIT_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (submitted)
        *submitted = s->submitted;
    if (completed)
        *completed = s->completed;
    if (pending)
        *pending = (int64_t)s->pending.size();
    if (bytes_in_use)
        *bytes_in_use = s->arena.used();
    if (peak_bytes)
        *peak_bytes = s->arena.peak();
    return SPLIT_OK;
}

int split_server_destroy(split_server *s)
{
    splitk::clear_error();
    if (!s)
        return SPLIT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable())
        s->worker.join();
    for (auto &kv : s->all)
        free_request(kv.second);
    for (auto &st : s->streams)
        (void)hipStreamDestroy(st);
    (void)hipFree(s->arena_base);
    delete s;
    return SPLIT_OK;
}

} // extern "C"
