// split_server.cpp -- served form: continuous batching of evaluation
// requests under an HBM budget, drained at tile granularity.
//
// Instances (a cost matrix and a demand scenario set) are registered once:
// the demands are copied into the server's device arena and stay resident,
// counted against the budget; the cost matrix stays on the host, where the
// tour constants of every request are computed.  A request is one giant
// tour evaluated on a resident instance, or one that brings its own
// instance (copied at admission and released at completion).
//
// The scheduler thread admits requests in arrival order while the arena,
// the job table and the queue have room (the paper's batching loop sizes
// its batches from free GPU memory, App. B; here admission against the
// arena plays that role and nothing is allocated per request).  Admission
// copies the request's tables into its arena block on the copy stream
// (from per-slot pinned staging), and a one-wave publish kernel appends the
// jobs to a device work queue.
// Drain kernels (split_serve.hip) take tiles from the queue; the scheduler
// keeps at most two drains per queue in flight and launches the next one
// while work remains.  The wave that finishes a job's last tile writes its
// result to pinned host memory, which the scheduler polls: no event or
// allocation per request.
//
// Reuse of device memory: a job has two arena blocks.  Its tables (and the
// demands of a request that brought its own instance), which drains read
// through the scalar and vector caches, are released with its table slot
// only once every drain that was running when it retired has ended, so no
// running drain can hold cached lines of memory that a later job reuses.
// Its costs and tour-ordered copy are released at retirement: drains never
// read the costs, and a drain wave reads only the tour-ordered rows it has
// just written itself (its own stores, made visible to the wave by a
// workgroup-scope fence), so stale lines of that memory are never read.
//
// The server's own reservation follows the paper's adaptive batching
// (App. B, Alg. "GPU-Based DP with Adaptive Batching"): the budget defaults
// to a share of free device memory, and a reservation that fails with
// out-of-memory is retried at half the size.

#include <hip/hip_runtime.h>

#include <algorithm>
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
#include "split_serve.h"

namespace {

using Clock = std::chrono::steady_clock;

#define sfail splitk::set_error

std::atomic<int> g_fail_allocs{0}; // test hook: device allocations to fail

// Device allocation through the failure hook.
hipError_t dev_alloc(void **p, size_t bytes)
{
    int n = g_fail_allocs.load();
    while (n > 0) {
        if (g_fail_allocs.compare_exchange_weak(n, n - 1))
            return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

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
        bytes = round(bytes);
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
        bytes = round(bytes);
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
    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t capacity() const { return cap_; }

  private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Instance {
    int64_t id = 0;
    int32_t N = 0;
    int64_t S = 0;
    std::vector<int32_t> dist;    // host copy, (N+1)^2
    std::vector<int16_t> h_dem;   // transient instances: demands until admission
    size_t off = 0, bytes = 0;    // arena block of the demands (bytes 0: not resident yet)
    int refs = 0;                 // requests referring to it
    bool transient = false;
    bool removed = false;
};

enum ReqState { PENDING, RUNNING, DONE };

struct Request {
    int64_t id = 0;
    Instance *inst = nullptr;
    int32_t n = 0, Q = 0;
    int32_t *costs_out = nullptr; // host, may be null
    // host-computed tour constants
    std::vector<int2> tab, ab;
    int32_t f0 = 0, bn = 0, variant = 0, pitch = 0;
    int32_t tiles = 0; // 64-scenario tiles
    bool ordered = false;
    // admission: tables block (released after the drains running at
    // retirement end) and outputs block (costs, tour-ordered copy: released
    // at retirement)
    size_t off = 0, bytes = 0;
    size_t off2 = 0, bytes2 = 0;
    int slot = -1;
    int32_t seq = 0;
    ReqState state = PENDING;
    Clock::time_point t_submit, t_done;
    int64_t sum = 0;
    double mean = 0.0;
    int error = SPLIT_OK;
};

// Memory released once the drains that were running at retirement have
// ended (drain ids below `mark` only).
struct Deferred {
    uint64_t mark;
    size_t off, bytes; // arena block (bytes 0: none)
    int slot;          // job slot (-1: none)
};

struct Drain {
    uint64_t id;
    int stream;
    hipEvent_t done;
    Clock::time_point launched;
    std::chrono::microseconds life; // how long its waves take tiles
};

} // namespace

struct split_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    int device = 0;
    int32_t max_len = 0;

    // device memory: fixed structures, then the arena
    char *dev_base = nullptr;
    splitk::ServeJob *d_jobs = nullptr;
    splitk::ServeQueue *d_queue[splitk::kServeQueues] = {}; // splitk::serve_queue order
    int *d_scratch = nullptr;
    uint32_t *d_scratch_mask = nullptr;
    char *arena_base = nullptr;
    Arena arena;

    // pinned host memory: results, per-slot staging (descriptor and tables)
    char *pin_base = nullptr;
    splitk::ServeResult *h_results = nullptr;
    char *h_stage = nullptr; // [kServeMaxJobs][stage_bytes]
    size_t stage_bytes = 0;

    hipStream_t copy_stream = nullptr, out_stream = nullptr;
    hipStream_t drain_stream[splitk::kServeQueues][2] = {};
    std::vector<hipEvent_t> event_pool;
    std::deque<Drain> drains[splitk::kServeQueues];
    int drain_rr[splitk::kServeQueues] = {};
    int drain_grid[splitk::kServeQueues] = {};
    uint64_t next_drain_id = 1;
    int64_t drains_launched = 0;
    int rate_khz = 100000; // device wall clock (ticks per ms) the drain waves read
    int64_t blocked = 0;        // scheduler rounds whose next request did not fit
    size_t deferred_bytes = 0;  // retired memory waiting for running drains to end
    hipEvent_t pub_event = nullptr; // recorded after the latest publish launch
    bool pub_recorded = false;
    splitk::ServeCtl ctl{};

    std::vector<int> free_slots;
    std::vector<Request *> slot_req; // [kServeMaxJobs]
    int32_t seq_counter = 0;
    int64_t outstanding[splitk::kServeQueues] = {}; // published, not finished, per queue
    int64_t backlog_tiles = 0; // tiles of admitted, unfinished requests
    std::deque<Request *> pending;
    std::vector<Request *> running;
    std::vector<Deferred> deferred;
    std::unordered_map<int64_t, Request *> all;
    std::unordered_map<int64_t, Instance *> instances;
    int64_t next_id = 1, next_inst = 1;
    int64_t submitted = 0, completed = 0;
    int failed = SPLIT_OK; // a HIP error stops all further device work
    char fail_text[256] = "";

    // ----- helpers (scheduler thread unless noted) -----
    size_t footprint_tables(const Request &r) const
    {
        const int64_t S = r.inst->S;
        size_t b = 0;
        b += a256(((size_t)r.n + splitk::kTabPad) * sizeof(int2)); // tab
        b += a256((size_t)std::max(r.n, 1) * sizeof(int2));        // ab
        b += a256(sizeof(splitk::TourRec));                         // rec
        if (r.inst->transient)
            b += a256((size_t)S * r.inst->N * 2);                 // own demands
        return b;
    }

    size_t footprint(const Request &r) const
    {
        return Arena::round(footprint_tables(r)) + Arena::round(footprint_outputs(r));
    }

    size_t footprint_outputs(const Request &r) const
    {
        const int64_t S = r.inst->S;
        size_t b = a256((size_t)S * 4);                             // costs
        if (r.ordered)
            b += a256((size_t)S * (size_t)r.pitch);               // tour-ordered copy
        return b;
    }

    uint64_t min_running_drain() const
    {
        uint64_t m = next_drain_id;
        for (int q = 0; q < splitk::kServeQueues; ++q)
            for (const Drain &d : drains[q])
                m = std::min(m, d.id);
        return m;
    }

    void fail_all(const char *what, hipError_t e)
    {
        if (failed == SPLIT_OK) {
            failed = SPLIT_EDEVICE;
            snprintf(fail_text, sizeof(fail_text), "%s: %s", what, hipGetErrorString(e));
        }
    }

    // Admits one request: staging and copies.  Returns false when
    // resources are short (the request stays pending).
    bool admit(Request *r, std::vector<Request *> &batch)
    {
        if (free_slots.empty())
            return false;
        const int qi = splitk::serve_queue(r->ordered, r->variant);
        if (outstanding[qi] >= splitk::kServeQueueCap - 2)
            return false;
        const size_t bytes = footprint_tables(*r), bytes2 = footprint_outputs(*r);
        size_t off = 0, off2 = 0;
        if (!arena.alloc(bytes, &off))
            return false;
        if (!arena.alloc(bytes2, &off2)) {
            arena.release(off, bytes);
            return false;
        }
        r->off = off;
        r->bytes = bytes;
        r->off2 = off2;
        r->bytes2 = bytes2;
        r->slot = free_slots.back();
        free_slots.pop_back();
        slot_req[r->slot] = r;
        r->seq = ++seq_counter;
        if (seq_counter >= (1 << 30))
            seq_counter = 0;

        Instance *in = r->inst;
        const int64_t S = in->S;
        char *blk = arena_base + off;
        size_t o = 0;
        int2 *d_tab = reinterpret_cast<int2 *>(blk + o);
        o += a256(((size_t)r->n + splitk::kTabPad) * sizeof(int2));
        int2 *d_ab = reinterpret_cast<int2 *>(blk + o);
        o += a256((size_t)std::max(r->n, 1) * sizeof(int2));
        splitk::TourRec *d_rec = reinterpret_cast<splitk::TourRec *>(blk + o);
        o += a256(sizeof(splitk::TourRec));
        char *blk2 = arena_base + off2;
        int32_t *d_costs = reinterpret_cast<int32_t *>(blk2);
        uint8_t *d_perm = r->ordered ? reinterpret_cast<uint8_t *>(blk2 + a256((size_t)S * 4))
                                     : nullptr;
        const int16_t *d_dem = nullptr;
        if (in->transient) {
            int16_t *dd = reinterpret_cast<int16_t *>(blk + o);
            o += a256((size_t)S * in->N * 2);
            hipError_t e = hipMemcpyAsync(dd, in->h_dem.data(), (size_t)S * in->N * 2,
                                          hipMemcpyHostToDevice, copy_stream);
            if (e != hipSuccess) {
                fail_all("copy demands", e);
                return true;
            }
            in->h_dem.clear();
            in->h_dem.shrink_to_fit();
            d_dem = dd;
        } else {
            d_dem = reinterpret_cast<const int16_t *>(arena_base + in->off);
        }

        // pinned staging of this slot: the job descriptor, then tab, ab, rec
        // laid out as in the arena block (the round's admit launch copies
        // them; the drain wave that runs a tile writes its tour-ordered rows)
        char *st = h_stage + (size_t)r->slot * stage_bytes + splitk::kStageHead;
        const size_t tab_b = ((size_t)r->n + splitk::kTabPad) * sizeof(int2);
        const size_t ab_b = (size_t)r->n * sizeof(int2);
        memcpy(st, r->tab.data(), tab_b);
        memcpy(st + a256(tab_b), r->ab.data(), ab_b);
        splitk::TourRec rec{};
        rec.n = r->n;
        rec.f0 = r->f0;
        rec.bn = r->bn;
        rec.status = 0;
        rec.maxc = 0;
        memcpy(st + a256(tab_b) + a256((size_t)std::max(r->n, 1) * sizeof(int2)), &rec,
               sizeof(rec));
        const size_t head_b = a256(tab_b) + a256((size_t)std::max(r->n, 1) * sizeof(int2)) +
                              sizeof(splitk::TourRec);
        (void)d_rec;
        splitk::ServeJob j{};
        j.demands = d_dem;
        j.perm = d_perm;
        j.tab = d_tab;
        j.ab = d_ab;
        j.costs = d_costs;
        j.S = S;
        j.N = in->N;
        j.n = r->n;
        j.Q = r->Q;
        j.f0 = r->f0;
        j.bn = r->bn;
        j.tiles = (int32_t)splitk::num_tiles(S);
        j.parts_done = splitk::kServeParts - std::min<int32_t>(splitk::kServeParts, j.tiles);
        // tiles per claim: one while the device is not saturated (every
        // tile of a lone request runs in parallel), up to kServeChunkMax
        // when the backlog holds several tiles per drain wave (fewer claims
        // and completion updates per tile)
        r->tiles = j.tiles;
        backlog_tiles += j.tiles;
        j.chunk = (int32_t)std::min<int64_t>(
            splitk::kServeChunkMax,
            std::max<int64_t>(1, backlog_tiles / (2 * (int64_t)drain_grid[qi])));
        j.variant = r->variant;
        j.pitch = r->pitch;
        j.seq = r->seq;
        j.head_bytes = (int32_t)head_b;
        memcpy(h_stage + (size_t)r->slot * stage_bytes, &j, sizeof(j));
        batch.push_back(r);
        return true;
    }

    // The round's launches on the copy stream, after any demand copies of
    // its requests: admit (tables and descriptors), then publish (queue
    // append), at most kPublishMax jobs per group.
    void publish(std::vector<Request *> &batch)
    {
        if (batch.empty() || failed)
            return;
        for (size_t i = 0; i < batch.size(); i += splitk::kPublishMax) {
            const int cnt = (int)std::min(batch.size() - i, (size_t)splitk::kPublishMax);
            splitk::AdmitBatch ab{};
            splitk::PublishBatch pb{};
            ab.count = cnt;
            pb.count = cnt;
            for (int k = 0; k < cnt; ++k) {
                const Request *r = batch[i + k];
                ab.slot[k] = r->slot;
                pb.entry[k] = r->slot | (splitk::serve_queue(r->ordered, r->variant) << 28);
            }
            hipError_t e = splitk::serve_launch_admit(d_jobs, h_stage, stage_bytes, ab, copy_stream);
            if (e != hipSuccess) {
                fail_all("admit launch", e);
                return;
            }
            splitk::ServeQueues qs{};
            for (int q = 0; q < splitk::kServeQueues; ++q)
                qs.q[q] = d_queue[q];
            e = splitk::serve_launch_publish(qs, pb, copy_stream);
            if (e != hipSuccess) {
                fail_all("publish launch", e);
                return;
            }
        }
        hipError_t e = hipEventRecord(pub_event, copy_stream);
        if (e != hipSuccess) {
            fail_all("publish event", e);
            return;
        }
        pub_recorded = true;
        for (Request *r : batch) {
            outstanding[splitk::serve_queue(r->ordered, r->variant)]++;
            r->state = RUNNING;
            running.push_back(r);
        }
        batch.clear();
    }

    hipEvent_t get_event()
    {
        if (event_pool.empty())
            return nullptr;
        hipEvent_t e = event_pool.back();
        event_pool.pop_back();
        return e;
    }

    void manage_drains(Clock::time_point now)
    {
        for (int qi = 0; qi < splitk::kServeQueues; ++qi) {
            // retire finished drains
            while (!drains[qi].empty()) {
                Drain &d = drains[qi].front();
                const hipError_t q = hipEventQuery(d.done);
                if (q == hipErrorNotReady)
                    break;
                if (q != hipSuccess)
                    fail_all("drain", q);
                event_pool.push_back(d.done);
                drains[qi].pop_front();
            }
            if (failed || outstanding[qi] == 0)
                continue;
            const bool none = drains[qi].empty();
            // the next drain is launched once the running one has stopped
            // taking tiles (its life is over), so its workgroups take the
            // slots the old one's waves free as they finish
            const bool aging =
                drains[qi].size() == 1 && now - drains[qi].back().launched > drains[qi].back().life;
            if (!none && !aging)
                continue;
            hipEvent_t ev = get_event();
            if (!ev)
                continue;
            const int si = drain_rr[qi]++ & 1;
            hipStream_t st = drain_stream[qi][si];
            // the drain starts after the latest publication has landed
            hipError_t e = pub_recorded ? hipStreamWaitEvent(st, pub_event, 0) : hipSuccess;
            // Drain life by backlog: with several tiles per drain wave queued
            // (saturation) a drain takes tiles for 24 ms and waits 200 us for
            // more, since each change of drain costs the device the tail of
            // the old drain's last tiles and a drain's stream keeps later
            // launches that share its hardware queue waiting until it ends;
            // longer lives hold retired jobs' tables (released only after the
            // drains running at retirement end) and with them admission.
            // Otherwise 1 ms and 20 us, so a light stream's launches and
            // retired memory do not wait long.
            const bool busy = backlog_tiles > 4 * (int64_t)drain_grid[qi];
            const auto life = std::chrono::microseconds(busy ? 24000 : 1000);
            splitk::ServeCtl c = ctl;
            c.life_ticks = (long long)rate_khz * (busy ? 24 : 1);
            c.idle_ticks = (long long)rate_khz / (busy ? 5 : 50);
            if (e == hipSuccess)
                e = splitk::serve_launch_drain(qi, c, d_queue[qi], drain_grid[qi], st);
            if (e == hipSuccess)
                e = hipEventRecord(ev, st);
            if (e != hipSuccess) {
                event_pool.push_back(ev);
                fail_all("drain launch", e);
                continue;
            }
            drains[qi].push_back(Drain{next_drain_id++, si, ev, now, life});
            drains_launched++;
        }
    }

    // Polls finished jobs (results in pinned memory).  Called unlocked; the
    // request objects it touches are owned by the scheduler while RUNNING.
    void collect(std::vector<Request *> &done)
    {
        for (size_t i = 0; i < running.size();) {
            Request *r = running[i];
            const splitk::ServeResult *res = h_results + r->slot;
            const int32_t seq = __atomic_load_n(&res->seq, __ATOMIC_ACQUIRE);
            if (seq != r->seq) {
                ++i;
                continue;
            }
            r->sum = res->sum;
            r->mean = res->mean;
            if (res->flags & 1)
                r->error = SPLIT_EINVAL;
            else if (res->flags)
                r->error = SPLIT_EDEVICE;
            if (r->costs_out && r->error == SPLIT_OK) {
                const char *d_costs = arena_base + r->off2;
                hipError_t e = hipMemcpyAsync(r->costs_out, d_costs, (size_t)r->inst->S * 4,
                                              hipMemcpyDeviceToHost, out_stream);
                if (e == hipSuccess)
                    e = hipStreamSynchronize(out_stream);
                if (e != hipSuccess) {
                    r->error = SPLIT_EDEVICE;
                    fail_all("copy costs", e);
                }
            }
            r->t_done = Clock::now();
            outstanding[splitk::serve_queue(r->ordered, r->variant)]--;
            backlog_tiles -= r->tiles;
            done.push_back(r);
            running[i] = running.back();
            running.pop_back();
        }
    }

    void release_deferred()
    {
        const uint64_t m = min_running_drain();
        for (size_t i = 0; i < deferred.size();) {
            if (deferred[i].mark <= m) {
                if (deferred[i].bytes) {
                    arena.release(deferred[i].off, deferred[i].bytes);
                    deferred_bytes -= Arena::round(deferred[i].bytes);
                }
                if (deferred[i].slot >= 0) {
                    slot_req[deferred[i].slot] = nullptr;
                    free_slots.push_back(deferred[i].slot);
                }
                deferred[i] = deferred.back();
                deferred.pop_back();
            } else {
                ++i;
            }
        }
    }

    void retire(Request *r)
    {
        // outputs: no drain reads them any more (every tile is done)
        if (r->bytes2)
            arena.release(r->off2, r->bytes2);
        r->bytes2 = 0;
        // tables: every drain launched so far may have touched them
        deferred.push_back(Deferred{next_drain_id, r->off, r->bytes, r->slot});
        deferred_bytes += Arena::round(r->bytes);
        Instance *in = r->inst;
        in->refs--;
        if (in->transient) {
            all_instances_erase(in);
        } else if (in->removed && in->refs == 0 && in->bytes) {
            deferred.push_back(Deferred{next_drain_id, in->off, in->bytes, -1});
            deferred_bytes += Arena::round(in->bytes);
            all_instances_erase(in);
        }
        r->inst = nullptr;
        r->state = DONE;
        completed++;
    }

    void all_instances_erase(Instance *in)
    {
        instances.erase(in->id);
        delete in;
    }

    void loop()
    {
        (void)hipSetDevice(device);
        std::vector<Request *> batch, done;
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            const auto now = Clock::now();
            bool progress = false;
            // completions (pinned memory reads only)
            done.clear();
            collect(done);
            for (Request *r : done)
                retire(r);
            if (!done.empty()) {
                progress = true;
                cv_done.notify_all();
            }
            manage_drains(now);
            release_deferred();
            // admission in arrival order
            while (!pending.empty() && !failed) {
                Request *r = pending.front();
                if (!admit(r, batch)) {
                    blocked++;
                    break;
                }
                pending.pop_front();
                progress = true;
            }
            publish(batch);
            manage_drains(Clock::now());
            if (failed) {
                // no further device work: every open request fails
                for (Request *r : pending) {
                    r->error = SPLIT_EDEVICE;
                    r->state = DONE;
                    if (--r->inst->refs == 0 && r->inst->transient)
                        all_instances_erase(r->inst);
                    r->inst = nullptr;
                    completed++;
                }
                pending.clear();
                for (Request *r : running) {
                    r->error = SPLIT_EDEVICE;
                    r->state = DONE;
                    completed++;
                }
                running.clear();
                cv_done.notify_all();
            }
            if (stop && pending.empty() && running.empty())
                break;
            if (!progress) {
                if (running.empty() && pending.empty()) {
                    bool drains_left = !deferred.empty();
                    for (int q = 0; q < splitk::kServeQueues; ++q)
                        drains_left = drains_left || !drains[q].empty();
                    if (drains_left)
                        cv_work.wait_for(lk, std::chrono::microseconds(200));
                    else
                        cv_work.wait(lk, [&] { return stop || !pending.empty(); });
                } else {
                    lk.unlock();
                    std::this_thread::sleep_for(std::chrono::microseconds(5));
                    lk.lock();
                }
            }
        }
        // wait for the drains to end before memory is released
        for (int qi = 0; qi < splitk::kServeQueues; ++qi)
            for (Drain &d : drains[qi]) {
                (void)hipEventSynchronize(d.done);
                event_pool.push_back(d.done);
            }
        for (int qi = 0; qi < splitk::kServeQueues; ++qi)
            drains[qi].clear();
    }
};

namespace {

// Tour constants on the host (the prep kernel's arithmetic for one tour):
// tab[j] = {sigma_j - 1, c_j}, ab[k-1] = {a_k, b_k}; validation as
// split_eval's host form.
int prepare(Request *r, const int32_t *tour, int32_t n, const Instance &in, int32_t Q)
{
    const int32_t N = in.N;
    int32_t lens[1] = {n};
    int32_t max_len = 0;
    int64_t total = 0;
    int rc = splitk::check_tours_host(tour, lens, 1, in.dist.data(), N, &max_len, &total);
    if (rc)
        return rc;
    const int64_t N1 = (int64_t)N + 1;
    const int32_t *dist = in.dist.data();
    r->n = n;
    r->Q = Q;
    r->tab.assign((size_t)n + splitk::kTabPad, int2{0, 0});
    r->ab.assign((size_t)std::max(n, 1), int2{0, 0});
    int64_t D = 0;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t c = tour[k];
        const int64_t out = dist[c], in_ = dist[(int64_t)c * N1];
        int64_t ck = 0, arc = 0;
        if (k + 1 < n) {
            const int32_t cn = tour[k + 1];
            arc = dist[(int64_t)c * N1 + cn];
            ck = in_ + dist[cn] - arc;
        }
        r->tab[(size_t)k + 1] = int2{c - 1, (int)ck};
        r->ab[(size_t)k] = int2{(int)(out - D), (int)(D + in_)};
        D += arc;
    }
    r->f0 = n > 0 ? dist[tour[0]] : 0;
    r->bn = n > 0 ? r->ab[(size_t)n - 1].y : 0;
    r->variant = Q > 200 ? splitk::SV_R64_16 : Q > 100 ? splitk::SV_R32_8 : splitk::SV_R32_6;
    r->ordered = N > splitk::kServeFusedMaxN;
    r->pitch = r->ordered ? splitk::ordered_pitch(n) : 0;
    return SPLIT_OK;
}

int enqueue(split_server *s, Request *r, int64_t *id)
{
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            r->inst->refs--;
            delete r;
            return sfail(SPLIT_EINVAL, "server is shutting down");
        }
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

} // namespace

extern "C" {

int split_debug_fail_allocations(int32_t count)
{
    splitk::clear_error();
    if (count < 0)
        return sfail(SPLIT_EINVAL, "count must be >= 0");
    g_fail_allocs.store(count);
    return SPLIT_OK;
}

int split_server_create(split_server **out, size_t budget_bytes, int32_t max_len)
{
    splitk::clear_error();
    if (!out || max_len < 1 || max_len > splitk::kMaxLen)
        return sfail(SPLIT_EINVAL, "need an output pointer and 1 <= max_len <= %d", splitk::kMaxLen);
    split_server *s = new split_server();
    s->max_len = max_len;
    auto bail = [&](int code, const char *what, hipError_t e) {
        if (s->dev_base)
            (void)hipFree(s->dev_base);
        if (s->pin_base)
            (void)hipHostFree(s->pin_base);
        for (hipEvent_t ev : s->event_pool)
            (void)hipEventDestroy(ev);
        if (s->pub_event)
            (void)hipEventDestroy(s->pub_event);
        for (hipStream_t st : {s->copy_stream, s->out_stream})
            if (st)
                (void)hipStreamDestroy(st);
        for (int q = 0; q < splitk::kServeQueues; ++q)
            for (hipStream_t st : s->drain_stream[q])
                if (st)
                    (void)hipStreamDestroy(st);
        delete s;
        return sfail(code, "%s: %s", what, hipGetErrorString(e));
    };
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess)
        return bail(SPLIT_EDEVICE, "no device", e);

    // fixed device structures
    const size_t jobs_b = a256(sizeof(splitk::ServeJob) * splitk::kServeMaxJobs);
    const size_t queue_b = a256(sizeof(splitk::ServeQueue));
    const size_t scratch_b =
        a256((size_t)splitk::kServeScratchSlots * splitk::kTile * ((size_t)max_len + 1) * 4);
    const size_t fixed = jobs_b + splitk::kServeQueues * queue_b + scratch_b + 256;
    size_t budget = budget_bytes;
    if (budget == 0) { // a share of free device memory (adaptive batch size)
        size_t fr = 0, tot = 0;
        e = hipMemGetInfo(&fr, &tot);
        if (e != hipSuccess)
            return bail(SPLIT_EDEVICE, "memory info", e);
        budget = fr / 4 * 3;
    }
    const size_t floor_b = (size_t)64 << 20;
    if (budget < floor_b + fixed)
        budget = floor_b + fixed;
    // reserve, halving on out-of-memory down to the floor
    for (;;) {
        e = dev_alloc(reinterpret_cast<void **>(&s->dev_base), budget);
        if (e == hipSuccess)
            break;
        (void)hipGetLastError();
        if (e != hipErrorOutOfMemory || budget / 2 < floor_b + fixed)
            return bail(SPLIT_ENOMEM, "cannot reserve device memory", e);
        budget /= 2;
    }
    char *p = s->dev_base;
    s->d_jobs = reinterpret_cast<splitk::ServeJob *>(p);
    p += jobs_b;
    for (int q = 0; q < splitk::kServeQueues; ++q) {
        s->d_queue[q] = reinterpret_cast<splitk::ServeQueue *>(p);
        p += queue_b;
    }
    s->d_scratch = reinterpret_cast<int *>(p);
    p += scratch_b;
    s->d_scratch_mask = reinterpret_cast<uint32_t *>(p);
    p += 256;
    s->arena_base = p;
    s->arena.init(budget - fixed);
    e = hipMemset(s->dev_base, 0, fixed);
    if (e != hipSuccess)
        return bail(SPLIT_EDEVICE, "clear server structures", e);

    // pinned host memory: results, per-slot staging
    s->stage_bytes = a256(sizeof(splitk::ServeJob)) +
                     a256(((size_t)max_len + splitk::kTabPad) * sizeof(int2)) +
                     a256((size_t)max_len * sizeof(int2)) + a256(sizeof(splitk::TourRec));
    const size_t res_b = a256(sizeof(splitk::ServeResult) * splitk::kServeMaxJobs);
    const size_t pin = res_b + s->stage_bytes * splitk::kServeMaxJobs;
    e = hipHostMalloc(reinterpret_cast<void **>(&s->pin_base), pin, hipHostMallocCoherent);
    if (e != hipSuccess)
        return bail(SPLIT_ENOMEM, "pinned host memory", e);
    memset(s->pin_base, 0, res_b);
    char *h = s->pin_base;
    s->h_results = reinterpret_cast<splitk::ServeResult *>(h);
    h += res_b;
    s->h_stage = h;

    e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&s->out_stream, hipStreamNonBlocking);
    for (int q = 0; q < splitk::kServeQueues && e == hipSuccess; ++q)
        for (int k = 0; k < 2 && e == hipSuccess; ++k)
            e = hipStreamCreateWithFlags(&s->drain_stream[q][k], hipStreamNonBlocking);
    if (e != hipSuccess)
        return bail(SPLIT_EDEVICE, "stream creation", e);
    for (int k = 0; k < 4 * splitk::kServeQueues && e == hipSuccess; ++k) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess)
            s->event_pool.push_back(ev);
    }
    if (e != hipSuccess)
        return bail(SPLIT_EDEVICE, "event creation", e);
    for (int q = 0; q < splitk::kServeQueues; ++q) {
        s->drain_grid[q] = splitk::serve_drain_grid(q, s->max_len);
        if (s->drain_grid[q] < 1)
            return bail(SPLIT_EDEVICE, "drain occupancy", hipGetLastError());
    }
    s->ctl.jobs = s->d_jobs;
    s->ctl.results = s->h_results;
    s->ctl.scratch = s->d_scratch;
    s->ctl.scratch_mask = s->d_scratch_mask;
    s->ctl.max_len = max_len;
    int rate_khz = 0; // the device wall clock the drain waves read
    e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, s->device);
    if (e != hipSuccess || rate_khz <= 0)
        rate_khz = 100000;
    s->rate_khz = rate_khz;
    // per launch the scheduler sets a drain's life and idle time by the
    // backlog (manage_drains); these are the light-load values
    s->ctl.idle_ticks = (long long)rate_khz / 50; // 20 us
    s->ctl.life_ticks = (long long)rate_khz;      // 1 ms
    e = hipEventCreateWithFlags(&s->pub_event, hipEventDisableTiming);
    if (e != hipSuccess)
        return bail(SPLIT_EDEVICE, "event creation", e);
    s->slot_req.assign(splitk::kServeMaxJobs, nullptr);
    for (int k = splitk::kServeMaxJobs - 1; k >= 0; --k)
        s->free_slots.push_back(k);
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return SPLIT_OK;
}

int split_server_add_instance(split_server *s, const int32_t *dist, int32_t N,
                              const int16_t *demands, int64_t S, int64_t *instance_id)
{
    splitk::clear_error();
    if (!s || !dist || !demands || !instance_id)
        return sfail(SPLIT_EINVAL, "null argument");
    if (N < 1 || N >= 65535 || S < 1)
        return sfail(SPLIT_EINVAL, "need 1 <= N < 65535 and S >= 1 (got N=%d S=%lld)", N,
                     (long long)S);
    Instance *in = new Instance();
    in->N = N;
    in->S = S;
    in->dist.assign(dist, dist + ((size_t)N + 1) * ((size_t)N + 1));
    const size_t bytes = a256((size_t)S * N * 2);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->failed) {
            delete in;
            return sfail(s->failed, "server failed: %s", s->fail_text);
        }
        if (bytes > s->arena.capacity()) {
            delete in;
            return sfail(SPLIT_ENOMEM, "instance needs %zu bytes, the budget holds %zu", bytes,
                         s->arena.capacity());
        }
        if (!s->arena.alloc(bytes, &in->off)) {
            delete in;
            return sfail(SPLIT_EAGAIN, "no room for the instance now (%zu bytes in use)",
                         s->arena.used());
        }
        in->bytes = bytes;
        in->id = s->next_inst++;
        s->instances[in->id] = in;
    }
    // the block was free and no running drain touched it since it was freed
    hipError_t e = hipMemcpy(s->arena_base + in->off, demands, (size_t)S * N * 2,
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->arena.release(in->off, in->bytes);
        s->instances.erase(in->id);
        delete in;
        return sfail(SPLIT_EDEVICE, "copy demands: %s", hipGetErrorString(e));
    }
    *instance_id = in->id;
    return SPLIT_OK;
}

int split_server_remove_instance(split_server *s, int64_t instance_id)
{
    splitk::clear_error();
    if (!s)
        return sfail(SPLIT_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->instances.find(instance_id);
    if (it == s->instances.end() || it->second->transient || it->second->removed)
        return sfail(SPLIT_EINVAL, "unknown instance %lld", (long long)instance_id);
    Instance *in = it->second;
    in->removed = true;
    if (in->refs == 0) {
        s->deferred.push_back(Deferred{s->next_drain_id, in->off, in->bytes, -1});
        s->deferred_bytes += Arena::round(in->bytes);
        s->instances.erase(it);
        delete in;
    }
    s->cv_work.notify_one();
    return SPLIT_OK;
}

int split_server_submit(split_server *s, int64_t instance_id, const int32_t *tour, int32_t n,
                        int32_t Q, int32_t *costs_out, int64_t *id)
{
    splitk::clear_error();
    if (!s || !id || (n > 0 && !tour))
        return sfail(SPLIT_EINVAL, "null argument");
    if (n < 0 || n > s->max_len || Q < 0)
        return sfail(SPLIT_EINVAL, "need 0 <= n <= %d and Q >= 0 (got n=%d Q=%d)", s->max_len, n,
                     Q);
    Instance *in = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->instances.find(instance_id);
        if (it == s->instances.end() || it->second->removed || it->second->transient)
            return sfail(SPLIT_EINVAL, "unknown instance %lld", (long long)instance_id);
        in = it->second;
        in->refs++; // held until the request retires
    }
    Request *r = new Request();
    r->inst = in;
    r->costs_out = costs_out;
    const int rc = prepare(r, tour, n, *in, Q);
    if (rc != SPLIT_OK) {
        std::lock_guard<std::mutex> lk(s->mu);
        in->refs--;
        delete r;
        return rc;
    }
    if (s->footprint(*r) > s->arena.capacity()) {
        std::lock_guard<std::mutex> lk(s->mu);
        in->refs--;
        const size_t need = s->footprint(*r);
        delete r;
        return sfail(SPLIT_ENOMEM, "request needs %zu bytes, the budget holds %zu", need,
                     s->arena.capacity());
    }
    return enqueue(s, r, id);
}

int split_server_submit_copy(split_server *s, const int32_t *tour, int32_t n, const int32_t *dist,
                             int32_t N, const int16_t *demands, int64_t S, int32_t Q,
                             int32_t *costs_out, int64_t *id)
{
    splitk::clear_error();
    if (!s || !id || !dist || !demands || (n > 0 && !tour))
        return sfail(SPLIT_EINVAL, "null argument");
    if (n < 0 || n > s->max_len || Q < 0 || N < 1 || N >= 65535 || S < 1)
        return sfail(SPLIT_EINVAL, "bad sizes n=%d N=%d S=%lld Q=%d", n, N, (long long)S, Q);
    Instance *in = new Instance();
    in->N = N;
    in->S = S;
    in->transient = true;
    in->refs = 1;
    in->dist.assign(dist, dist + ((size_t)N + 1) * ((size_t)N + 1));
    Request *r = new Request();
    r->inst = in;
    r->costs_out = costs_out;
    const int rc = prepare(r, tour, n, *in, Q);
    if (rc != SPLIT_OK) {
        delete r;
        delete in;
        return rc;
    }
    const size_t need = s->footprint(*r);
    if (need > s->arena.capacity()) {
        delete r;
        delete in;
        return sfail(SPLIT_ENOMEM, "request needs %zu bytes, the budget holds %zu", need,
                     s->arena.capacity());
    }
    in->h_dem.assign(demands, demands + (size_t)S * N);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        in->id = -(s->next_inst++); // transient ids are negative (never looked up)
        s->instances[in->id] = in;
    }
    return enqueue(s, r, id);
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
    delete r;
    if (rc == SPLIT_EINVAL)
        return sfail(rc, "request %lld: negative demand found on the device", (long long)id);
    return rc == SPLIT_OK ? SPLIT_OK
                          : sfail(rc, "request %lld failed on the device", (long long)id);
}

int split_server_wait(split_server *s, int64_t id)
{
    splitk::clear_error();
    if (!s)
        return sfail(SPLIT_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->all.find(id) == s->all.end())
        return sfail(SPLIT_EINVAL, "unknown request id %lld", (long long)id);
    // the request is looked up again at every wake-up: another thread may
    // have polled (and freed) it meanwhile
    s->cv_done.wait(lk, [&] {
        auto it = s->all.find(id);
        return it == s->all.end() || it->second->state == DONE;
    });
    return SPLIT_OK;
}

int split_server_stats(split_server *s, split_server_stats_t *out)
{
    splitk::clear_error();
    if (!s || !out)
        return sfail(SPLIT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->pending = (int64_t)s->pending.size();
    out->running = (int64_t)s->running.size();
    out->bytes_in_use = s->arena.used();
    out->peak_bytes = s->arena.peak();
    out->capacity = s->arena.capacity();
    out->drains = s->drains_launched;
    out->deferred_bytes = s->deferred_bytes;
    out->blocked_rounds = s->blocked;
    out->instances = 0;
    for (auto &kv : s->instances)
        out->instances += kv.second->transient ? 0 : 1;
    return s->failed ? sfail(s->failed, "server failed: %s", s->fail_text) : SPLIT_OK;
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
    (void)hipStreamSynchronize(s->copy_stream);
    (void)hipDeviceSynchronize();
    for (auto &kv : s->all)
        delete kv.second;
    for (auto &kv : s->instances)
        delete kv.second;
    for (hipEvent_t ev : s->event_pool)
        (void)hipEventDestroy(ev);
    if (s->pub_event)
        (void)hipEventDestroy(s->pub_event);
    for (hipStream_t st : {s->copy_stream, s->out_stream})
        if (st)
            (void)hipStreamDestroy(st);
    for (int q = 0; q < splitk::kServeQueues; ++q)
        for (hipStream_t st : s->drain_stream[q])
            if (st)
                (void)hipStreamDestroy(st);
    (void)hipFree(s->dev_base);
    (void)hipHostFree(s->pin_base);
    delete s;
    return SPLIT_OK;
}

} // extern "C"
