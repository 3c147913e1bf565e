// split_serve.hip -- drain kernels of the served form: continuous batching at
// the granularity of a tile of 64 scenarios.
//
// Admitted requests become jobs in a device job table; their slots are
// appended to a work queue by a one-wave publish kernel that runs on the
// scheduler's copy stream right after the job's tables arrive.  A drain
// kernel is a grid of one-wave workgroups; every wave repeatedly takes the
// next tile of the job at the queue head (an atomic counter per job), runs
// the split recursion for its 64 scenarios (paper Sec. 2.3) and adds the
// tile's exact partial sum to the job.  When a job has no tiles left the
// waves advance the head to the next job, so tiles of jobs published while
// a drain runs join it at once and the work of consecutive requests
// overlaps on the device.  The wave that finishes a job's last tile folds
// the sum into the job's result (mean = sum / S, one IEEE double division)
// and writes it to host-visible memory, sequence number last.
//
// Every wave leaves once the queue has stayed empty for `idle_ticks`, and
// takes no new tile after `life_ticks`; the scheduler relaunches drains
// while work remains.  A tile whose windows leave the register ring, or
// whose demands do not fit a byte, runs the exact recursion inline with a
// value history from a small scratch pool.
//
// Two drains exist: the fused one stages the tile's rows in LDS (pools of
// at most kServeFusedMaxN customers); the ordered one streams each lane's
// row of the tour-ordered copy that a permute launch wrote at admission.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "split_device.h"
#include "split_dp.h"
#include "split_eval.h"
#include "split_internal.h"
#include "split_serve.h"

namespace splitk {

namespace {

template <typename T> __device__ __forceinline__ T ld_agent(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ long long ticks() { return (long long)wall_clock64(); }

// wave-uniform copies (every lane holds the same value; readfirstlane lets
// the compiler keep it in SGPRs, which the window blocks require)
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni64(int64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T> __device__ __forceinline__ T *uptr(T *p)
{
    return reinterpret_cast<T *>(uni64(reinterpret_cast<int64_t>(p)));
}

// A job's fields as the drain uses them (read once per tile, after the claim).
struct JobView {
    const int16_t *demands;
    const uint8_t *perm;
    const uint8_t *tile_bad;
    const int2 *tab;
    const int2 *ab;
    int32_t *costs;
    int64_t S;
    int N, n, Q, f0, bn, tiles, variant, pitch;
};

__device__ __forceinline__ JobView read_job(const ServeJob *j)
{
    JobView v;
    v.demands = uptr(ld_agent(&j->demands));
    v.perm = uptr(ld_agent(&j->perm));
    v.tile_bad = uptr(ld_agent(&j->tile_bad));
    v.tab = uptr(ld_agent(&j->tab));
    v.ab = uptr(ld_agent(&j->ab));
    v.costs = uptr(ld_agent(&j->costs));
    v.S = uni64(ld_agent(&j->S));
    v.N = uni(ld_agent(&j->N));
    v.n = uni(ld_agent(&j->n));
    v.Q = uni(ld_agent(&j->Q));
    v.f0 = uni(ld_agent(&j->f0));
    v.bn = uni(ld_agent(&j->bn));
    v.tiles = uni(ld_agent(&j->tiles));
    v.variant = uni(ld_agent(&j->variant));
    v.pitch = uni(ld_agent(&j->pitch));
    return v;
}

// Lane 0 takes the next tile from the queue; returns false (uniformly) when
// the wave should leave.
__device__ bool claim(ServeQueue *q, ServeJob *jobs, long long start, long long &idle_since,
                      const ServeCtl &ctl, int lane, int &slot, int &tile)
{
    int s_out = -1, t_out = -1, quit = 0;
    if (lane == 0) {
        for (;;) {
            const long long now = ticks();
            if (now - start > ctl.life_ticks) {
                quit = 1;
                break;
            }
            const uint32_t h = __hip_atomic_load(&q->head, __ATOMIC_ACQUIRE,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t t = __hip_atomic_load(&q->tail, __ATOMIC_ACQUIRE,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            if (h == t) {
                if (now - idle_since > ctl.idle_ticks) {
                    quit = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(16);
                continue;
            }
            const int s = ld_agent(&q->ring[h & (kServeQueueCap - 1)]);
            const int k = atomicAdd(&jobs[s].next_tile, 1);
            if (k < ld_agent(&jobs[s].tiles)) {
                s_out = s;
                t_out = k;
                break;
            }
            // no tiles left in this job: move the head on (another wave may
            // already have)
            uint32_t expect = h;
            __hip_atomic_compare_exchange_strong(&q->head, &expect, h + 1, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    quit = uni(__shfl(quit, 0, kWave));
    slot = uni(__shfl(s_out, 0, kWave));
    tile = uni(__shfl(t_out, 0, kWave));
    return !quit;
}

// Exact recursion for the rows of a tile, with a value history borrowed
// from the scratch pool (bounded wait; on time-out the tile's costs are
// SPLIT_INF and the job is flagged).
__device__ int exact_tile(const ServeCtl &ctl, const JobView &jv, int64_t s0, int rows, int lane,
                          bool &negq, bool &no_scratch)
{
    int bit = -1;
    if (lane == 0) {
        const long long t0 = ticks();
        while (bit < 0 && ticks() - t0 < 100LL * 1000 * 1000) { // one second at 100 MHz
            const uint32_t m = ld_agent(ctl.scratch_mask);
            const uint32_t freebits = ~m & ((1u << kServeScratchSlots) - 1u);
            if (freebits == 0) {
                __builtin_amdgcn_s_sleep(32);
                continue;
            }
            const int b = __builtin_ctz(freebits);
            const uint32_t old = atomicOr(ctl.scratch_mask, 1u << b);
            if (!(old & (1u << b)))
                bit = b;
        }
    }
    bit = uni(__shfl(bit, 0, kWave));
    if (bit < 0) {
        no_scratch = true;
        return kInf;
    }
    int *V = ctl.scratch + (int64_t)bit * kWave * (ctl.max_len + 1);
    int v = kInf;
    if (lane < rows)
        v = exact_lane(jv.demands + (s0 + lane) * jv.N, jv.tab, jv.ab, jv.n, jv.Q, V, lane, negq);
    __threadfence(); // the history is complete before another wave may take the slot
    if (lane == 0)
        atomicAnd(ctl.scratch_mask, ~(1u << bit));
    return v;
}

template <bool ORDERED>
__device__ __forceinline__ int fast_tile(const JobView &jv, const uint8_t *lds, int64_t s0,
                                         int lane, int rows, bool &ovf)
{
    CInt *tab = (CInt *)jv.tab;
    int m = kInf;
    if (lane < rows) {
        if (ORDERED) {
            const uint8_t *row = jv.perm + (s0 + lane) * jv.pitch;
            switch (jv.variant) {
            case SV_R32_6:
                m = dp_lane_ordered<32, 6, 3, 3>(row, jv.pitch, tab, jv.n, jv.f0, jv.Q, ovf);
                break;
            case SV_R32_8:
                m = dp_lane_ordered<32, 8, 3, 3>(row, jv.pitch, tab, jv.n, jv.f0, jv.Q, ovf);
                break;
            default:
                m = dp_lane_ordered<64, 16, 4, 4>(row, jv.pitch, tab, jv.n, jv.f0, jv.Q, ovf);
                break;
            }
        } else {
            const uint8_t *row = lds + (int64_t)lane * jv.N;
            switch (jv.variant) {
            case SV_R32_6:
                m = dp_lane<32, 6, 3, 3>(row, tab, jv.n, jv.f0, jv.Q, ovf);
                break;
            case SV_R32_8:
                m = dp_lane<32, 8, 3, 3>(row, tab, jv.n, jv.f0, jv.Q, ovf);
                break;
            default:
                m = dp_lane<64, 16, 4, 4>(row, tab, jv.n, jv.f0, jv.Q, ovf);
                break;
            }
        }
    }
    return m + jv.bn;
}

template <bool ORDERED>
__device__ void run_tile(const ServeCtl &ctl, int slot, int tile, uint8_t *lds, int lane)
{
    ServeJob *job = ctl.jobs + slot;
    const JobView jv = read_job(job);
    const int64_t s0 = (int64_t)tile * kWave;
    const int rows = (int)min<int64_t>(kWave, jv.S - s0);
    bool negq = false, no_scratch = false;
    int v = 0;
    if (jv.n > 0) {
        bool ok;
        if (ORDERED) {
            ok = jv.tile_bad[tile] == 0;
        } else {
            int &s_bad = *reinterpret_cast<int *>(lds + (((size_t)kWave * kServeFusedMaxN + 15) &
                                                          ~(size_t)15));
            ok = stage_tile_u8(jv.demands + s0 * jv.N, lds, (int64_t)rows * jv.N, lane, kWave,
                               s_bad);
        }
        bool ovf = false;
        if (ok)
            v = fast_tile<ORDERED>(jv, lds, s0, lane, rows, ovf);
        if (!ok || ballot(ovf) != 0)
            v = exact_tile(ctl, jv, s0, rows, lane, negq, no_scratch);
    }
    const bool inf = lane < rows && (v >= kInf || no_scratch);
    const bool fin = lane < rows && !inf;
    if (lane < rows)
        jv.costs[s0 + lane] = inf ? SPLIT_INF : v;
    const long long sm = wave_sum_i64(fin ? (long long)v : 0LL);
    const int ni = wave_sum_i32(inf ? 1 : 0);
    const bool flag_neg = ballot(negq) != 0;
    if (lane == 0) {
        if (sm)
            atomicAdd(reinterpret_cast<unsigned long long *>(&job->sum), (unsigned long long)sm);
        if (ni)
            atomicAdd(reinterpret_cast<unsigned long long *>(&job->ninf), (unsigned long long)ni);
        if (flag_neg)
            atomicOr(&job->flags, 1);
        if (no_scratch)
            atomicOr(&job->flags, 2);
        __threadfence(); // costs and partial sums before the tile counts as done
        const int done = atomicAdd(&job->tiles_done, 1) + 1;
        if (done == jv.tiles) {
            __threadfence();
            const long long sum = (long long)atomicAdd(
                reinterpret_cast<unsigned long long *>(&job->sum), 0ull);
            const long long ninf = (long long)atomicAdd(
                reinterpret_cast<unsigned long long *>(&job->ninf), 0ull);
            const int flags = atomicOr(&job->flags, 0);
            ServeResult *r = ctl.results + slot;
            if (flags) {
                r->sum = SPLIT_SUM_INVALID;
                r->mean = __builtin_nan("");
            } else if (ninf) {
                r->sum = INT64_MAX;
                r->mean = __builtin_inf();
            } else {
                r->sum = sum;
                r->mean = (double)sum / (double)jv.S;
            }
            r->flags = flags;
            __threadfence_system();
            __hip_atomic_store(&r->seq, ld_agent(&job->seq), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

} // namespace

// grid of one-wave workgroups; LDS: the fused drain's tile (kServeFusedMaxN
// bytes per row) plus the staging flag
template <bool ORDERED>
__global__ __launch_bounds__(kWave) void serve_drain_kernel(ServeCtl ctl, ServeQueue *q)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const int lane = threadIdx.x;
    const long long start = ticks();
    long long idle_since = start;
    int slot, tile;
    while (claim(q, ctl.jobs, start, idle_since, ctl, lane, slot, tile)) {
        run_tile<ORDERED>(ctl, slot, tile, lds, lane);
        idle_since = ticks();
    }
}

// one wave: copy the batch's staged job descriptors (pinned host memory, at
// the start of each slot's staging area) into their table slots, then
// append the slots to their queues and publish the new tails with release
// order
__global__ __launch_bounds__(kWave) void serve_publish_kernel(ServeQueue *q0, ServeQueue *q1,
                                                              ServeJob *jobs,
                                                              const char *stage_base,
                                                              size_t stage_bytes,
                                                              PublishBatch batch)
{
    const int lane = threadIdx.x;
    constexpr int words = (int)(sizeof(ServeJob) / sizeof(uint32_t));
    for (int i = 0; i < batch.count; ++i) {
        const int s = batch.entry[i] & ((1 << 30) - 1);
        const uint32_t *src =
            reinterpret_cast<const uint32_t *>(stage_base + (size_t)s * stage_bytes);
        uint32_t *dst = reinterpret_cast<uint32_t *>(jobs + s);
        for (int w = lane; w < words; w += kWave)
            __hip_atomic_store(dst + w, src[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence();
    if (lane == 0) {
        uint32_t t0 = __hip_atomic_load(&q0->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t t1 = __hip_atomic_load(&q1->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t b0 = t0, b1 = t1;
        for (int i = 0; i < batch.count; ++i) {
            const int s = batch.entry[i] & ((1 << 30) - 1);
            if (batch.entry[i] >> 30)
                __hip_atomic_store(&q1->ring[t1++ & (kServeQueueCap - 1)], s, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            else
                __hip_atomic_store(&q0->ring[t0++ & (kServeQueueCap - 1)], s, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (t0 != b0)
            __hip_atomic_store(&q0->tail, t0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (t1 != b1)
            __hip_atomic_store(&q1->tail, t1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

static size_t drain_lds(bool ordered)
{
    return ordered ? 0 : (((size_t)kWave * kServeFusedMaxN + 15) & ~(size_t)15) + 16;
}

int serve_drain_grid(bool ordered)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const void *fn = ordered ? reinterpret_cast<const void *>(&serve_drain_kernel<true>)
                             : reinterpret_cast<const void *>(&serve_drain_kernel<false>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kWave, drain_lds(ordered)) !=
            hipSuccess ||
        per < 1)
        per = 1;
    return cus * per;
}

hipError_t serve_launch_drain(bool ordered, const ServeCtl &ctl, ServeQueue *q, int grid,
                              hipStream_t stream)
{
    if (ordered)
        hipLaunchKernelGGL(serve_drain_kernel<true>, dim3(grid), dim3(kWave), 0, stream, ctl, q);
    else
        hipLaunchKernelGGL(serve_drain_kernel<false>, dim3(grid), dim3(kWave), drain_lds(false),
                           stream, ctl, q);
    return hipGetLastError();
}

hipError_t serve_launch_publish(ServeQueue *q0, ServeQueue *q1, ServeJob *jobs,
                                const char *stage_base, size_t stage_bytes,
                                const PublishBatch &batch, hipStream_t stream)
{
    hipLaunchKernelGGL(serve_publish_kernel, dim3(1), dim3(kWave), 0, stream, q0, q1, jobs,
                       stage_base, stage_bytes, batch);
    return hipGetLastError();
}

} // namespace splitk
