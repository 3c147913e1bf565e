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
// at most kServeFusedMaxN customers); the ordered one first writes the
// tile's rows in tour order into the job's copy (gathered from the demand
// rows by the same wave) and then streams each lane's row of that copy.

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
// the wave should leave.  A wave caches the queue position it last read a
// job from (`cur_h`, its slot and tile count): only when the head has moved
// past it does the wave read the tail with acquire order (the publish
// kernel's release makes the job's descriptor and tables visible) and the
// new head job's slot, and `fresh` tells the caller to read the descriptor
// again.  Tiles are claimed from the partition `home` (the workgroup index
// modulo the partition count) first, then from the others in turn; a
// partition whose claim counter has passed its tile count is skipped with
// a load instead of an add.  When every partition of the head job is
// claimed the head moves on.
struct ClaimCache {
    uint32_t h;  // queue position of the cached job (valid when s >= 0)
    int s;       // its slot
    int tiles;   // its tile count
    int chunk;   // tiles per claim
};

__device__ bool claim(ServeQueue *q, ServeJob *jobs, long long start, long long &idle_since,
                      const ServeCtl &ctl, int lane, int home, ClaimCache &cc, int &slot,
                      int &tile, int &count, int &part, bool &fresh)
{
    int s_out = -1, t_out = -1, c_out = 0, p_out = -1, quit = 0, fr = 0;
    if (lane == 0) {
        for (;;) {
            const long long now = ticks();
            if (now - start > ctl.life_ticks) {
                quit = 1;
                break;
            }
            const uint32_t h = __hip_atomic_load(&q->head, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            if (cc.s < 0 || h != cc.h) {
                // relaxed: a job's descriptor and tables are written by
                // kernels that completed (and wrote back) before the publish
                // kernel stored the tail, and no cache of a running drain
                // holds lines of reused memory (memory is reused only after
                // every drain running at its retirement has ended), so the
                // reads below see them without an acquire's cache
                // invalidation
                const uint32_t t = __hip_atomic_load(&q->tail, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                if (h == t) {
                    if (now - idle_since > ctl.idle_ticks) {
                        quit = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(16);
                    continue;
                }
                cc.h = h;
                cc.s = ld_agent(&q->ring[h & (kServeQueueCap - 1)]);
                cc.tiles = ld_agent(&jobs[cc.s].tiles);
                cc.chunk = ld_agent(&jobs[cc.s].chunk);
                fr = 1;
            }
            ServeJob *jb = jobs + cc.s;
            for (int i = 0; i < kServeParts && s_out < 0; ++i) {
                const int p = (home + i) & (kServeParts - 1);
                const int lo = serve_part_lo(cc.tiles, p);
                const int cnt = serve_part_lo(cc.tiles, p + 1) - lo;
                if (cnt == 0 || ld_agent(&jb->part[p].next) >= cnt)
                    continue;
                const int k = atomicAdd(&jb->part[p].next, cc.chunk);
                if (k < cnt) {
                    s_out = cc.s;
                    t_out = lo + k;
                    c_out = min(cc.chunk, cnt - k);
                    p_out = p;
                }
            }
            if (s_out >= 0)
                break;
            // every partition claimed: move the head on (another wave may
            // already have)
            uint32_t expect = h;
            __hip_atomic_compare_exchange_strong(&q->head, &expect, h + 1, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    quit = uni(__shfl(quit, 0, kWave));
    slot = uni(__shfl(s_out, 0, kWave));
    tile = uni(__shfl(t_out, 0, kWave));
    count = uni(__shfl(c_out, 0, kWave));
    part = uni(__shfl(p_out, 0, kWave));
    fresh = uni(__shfl(fr, 0, kWave)) != 0;
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

// The tile's rows in tour order into the job's copy: byte j - 1 of row s is
// the demand of position j (zero from n to the pitch).  Returns false
// (uniformly) when a demand lies outside [0, 255].
//
// Pools of at most kServeStageMaxN customers: eight rows at a time are
// staged in LDS as bytes with 16-byte coalesced loads (all of a lane's
// chunks in flight together) and rewritten in tour order from there, so
// the gather runs on LDS.  Larger pools: consecutive lanes take consecutive
// 16-position chunks of one row straight from global memory (a load
// instruction touches a few lines of that row), two chunks per lane in
// flight.  cust: the tour's customer indices (LDS).
constexpr int kGatherChunks = 2;

__device__ __forceinline__ u32x4 pack16(const int (&v)[16], uint32_t &bad)
{
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t x = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int val = v[q * 4 + b];
            bad |= (uint32_t)val & 0xFFFFFF00u; // outside [0, 255]
            x |= ((uint32_t)val & 0xFFu) << (8 * b);
        }
        w[q] = x;
    }
    return u32x4{w[0], w[1], w[2], w[3]};
}

__device__ bool gather_tile(const JobView &jv, int64_t s0, int rows, const uint16_t *cust,
                            uint8_t *rowbuf, int &s_bad, int lane)
{
    const int chunks = jv.pitch / 16;
    uint8_t *dst = const_cast<uint8_t *>(jv.perm) + s0 * jv.pitch;
    uint32_t bad = 0;
    bool ok = true;
    if (jv.N <= kServeStageMaxN) {
        for (int rb0 = 0; rb0 < rows; rb0 += kServeStageRows) {
            const int rb = min(kServeStageRows, rows - rb0);
            // rows s0+rb0 .. start 16-byte aligned: s0 + rb0 is a multiple of 8
            ok = stage_tile_u8(jv.demands + (s0 + rb0) * jv.N, rowbuf, (int64_t)rb * jv.N, lane,
                               kWave, s_bad) && ok;
            for (int idx = lane; idx < rb * chunks; idx += kWave) {
                const int r = idx / chunks;
                const int c = idx - r * chunks;
                const uint8_t *row = rowbuf + r * jv.N;
                int w[16];
                if (c * 16 < jv.n) {
                    // the chunk's 16 customer indices in two 16-byte LDS reads
                    // (the tour array is zero-padded to a multiple of 16)
                    const u32x4 *cp = reinterpret_cast<const u32x4 *>(cust) + 2 * c;
                    const u32x4 c0 = cp[0], c1 = cp[1];
                    const uint32_t cw[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
                    for (int b = 0; b < 16; ++b) {
                        const int cu = (int)((cw[b >> 1] >> (16 * (b & 1))) & 0xFFFFu);
                        w[b] = c * 16 + b < jv.n ? row[cu] : 0;
                    }
                } else {
#pragma unroll
                    for (int b = 0; b < 16; ++b)
                        w[b] = 0; // past the tour: the row's zero padding
                }
                reinterpret_cast<u32x4 *>(dst + (int64_t)(rb0 + r) * jv.pitch)[c] = pack16(w, bad);
            }
            __syncthreads(); // the next batch overwrites the staged rows
        }
    } else {
        const int total = rows * chunks;
        for (int base = 0; base < total; base += kGatherChunks * kWave) {
            int v[kGatherChunks][16];
#pragma unroll
            for (int u = 0; u < kGatherChunks; ++u) {
                const int idx = base + u * kWave + lane;
                const int r = idx / chunks;
                const int c = idx - r * chunks;
                const int16_t *row = jv.demands + (s0 + r) * jv.N;
#pragma unroll
                for (int b = 0; b < 16; ++b) {
                    const int j = c * 16 + b;
                    v[u][b] = idx < total && j < jv.n ? row[cust[j]] : 0;
                }
            }
#pragma unroll
            for (int u = 0; u < kGatherChunks; ++u) {
                const int idx = base + u * kWave + lane;
                if (idx >= total)
                    continue;
                const int r = idx / chunks;
                const int c = idx - r * chunks;
                reinterpret_cast<u32x4 *>(dst + (int64_t)r * jv.pitch)[c] = pack16(v[u], bad);
            }
        }
    }
    // the stores complete before the recursion of this wave reads them back
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    return ok && ballot(bad != 0) == 0;
}

template <bool ORDERED, bool WIDE>
__device__ __forceinline__ int fast_tile(const JobView &jv, const uint8_t *lds, int64_t s0,
                                         int lane, int rows, bool &ovf)
{
    CInt *tab = (CInt *)jv.tab;
    int m = kInf;
    if (lane < rows) {
        if (ORDERED) {
            const uint8_t *row = jv.perm + (s0 + lane) * jv.pitch;
            if (WIDE)
                m = dp_lane_ordered<64, 16, 4, 4>(row, jv.pitch, tab, jv.n, jv.f0, jv.Q, ovf);
            else if (jv.variant == SV_R32_6)
                m = dp_lane_ordered<32, 6, 3, 3>(row, jv.pitch, tab, jv.n, jv.f0, jv.Q, ovf);
            else
                m = dp_lane_ordered<32, 8, 3, 3>(row, jv.pitch, tab, jv.n, jv.f0, jv.Q, ovf);
        } else {
            const uint8_t *row = lds + (int64_t)lane * jv.N;
            if (WIDE)
                m = dp_lane<64, 16, 4, 4>(row, tab, jv.n, jv.f0, jv.Q, ovf);
            else if (jv.variant == SV_R32_6)
                m = dp_lane<32, 6, 3, 3>(row, tab, jv.n, jv.f0, jv.Q, ovf);
            else
                m = dp_lane<32, 8, 3, 3>(row, tab, jv.n, jv.f0, jv.Q, ovf);
        }
    }
    return m + jv.bn;
}

// Partial results of the tiles a wave has run since its last claim.
struct TileAcc {
    long long sum; // exact sum of finite costs
    int ninf;      // SPLIT_INF costs
    bool neg;      // a negative demand was read
    bool no_scratch; // an exact tile found no value history in time
};

template <bool ORDERED, bool WIDE>
__device__ void run_tile(const ServeCtl &ctl, const JobView &jv, int tile, uint8_t *lds,
                         int lane, TileAcc &acc)
// (ordered drain: lds holds the tour's customer indices)
{
    const int64_t s0 = (int64_t)tile * kWave;
    const int rows = (int)min<int64_t>(kWave, jv.S - s0);
    bool negq = false, no_scratch = false;
    int v = 0;
    if (jv.n > 0) {
        bool ok;
        if (ORDERED) {
            const size_t cust_bytes = 2 * (((size_t)ctl.max_len + 15) & ~(size_t)15);
            uint8_t *rowbuf = lds + cust_bytes;
            int &s_bad = *reinterpret_cast<int *>(rowbuf + kServeStageRows * kServeStageMaxN);
            ok = gather_tile(jv, s0, rows, reinterpret_cast<const uint16_t *>(lds), rowbuf, s_bad,
                             lane);
        } else {
            int &s_bad = *reinterpret_cast<int *>(lds + (((size_t)kWave * kServeFusedMaxN + 15) &
                                                          ~(size_t)15));
            ok = stage_tile_u8(jv.demands + s0 * jv.N, lds, (int64_t)rows * jv.N, lane, kWave,
                               s_bad);
        }
        bool ovf = false;
        if (ok)
            v = fast_tile<ORDERED, WIDE>(jv, lds, s0, lane, rows, ovf);
        if (!ok || ballot(ovf) != 0)
            v = exact_tile(ctl, jv, s0, rows, lane, negq, no_scratch);
    }
    const bool inf = lane < rows && (v >= kInf || no_scratch);
    const bool fin = lane < rows && !inf;
    if (lane < rows)
        jv.costs[s0 + lane] = inf ? SPLIT_INF : v;
    acc.sum += wave_sum_i64(fin ? (long long)v : 0LL);
    acc.ninf += wave_sum_i32(inf ? 1 : 0);
    acc.neg = acc.neg || ballot(negq) != 0;
    acc.no_scratch = acc.no_scratch || no_scratch;
}

// The claimed tiles' partial sums into their partition, then the
// partition's and the job's completion counts; the wave that completes the
// job folds the partitions and writes the result to host-visible memory.
__device__ void finish_chunk(const ServeCtl &ctl, const JobView &jv, int slot, int part,
                             int count, const TileAcc &acc, int lane)
{
    if (lane != 0)
        return;
    ServeJob *job = ctl.jobs + slot;
    ServePart &pt = job->part[part];
    if (acc.sum)
        atomicAdd(reinterpret_cast<unsigned long long *>(&pt.sum), (unsigned long long)acc.sum);
    if (acc.ninf)
        atomicAdd(reinterpret_cast<unsigned long long *>(&pt.ninf), (unsigned long long)acc.ninf);
    if (acc.neg)
        atomicOr(&job->flags, 1);
    if (acc.no_scratch)
        atomicOr(&job->flags, 2);
    __threadfence(); // costs and partial sums before the tiles count as done
    const int cnt = serve_part_lo(jv.tiles, part + 1) - serve_part_lo(jv.tiles, part);
    if (atomicAdd(&pt.done, count) + count != cnt)
        return;
    __threadfence(); // the partition's sums before it counts as done
    if (atomicAdd(&job->parts_done, 1) + 1 != kServeParts)
        return;
    __threadfence();
    long long sum = 0, ninf = 0;
    for (int p = 0; p < kServeParts; ++p) {
        sum += (long long)atomicAdd(reinterpret_cast<unsigned long long *>(&job->part[p].sum),
                                    0ull);
        ninf += (long long)atomicAdd(reinterpret_cast<unsigned long long *>(&job->part[p].ninf),
                                     0ull);
    }
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
    __hip_atomic_store(&r->seq, ld_agent(&job->seq), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

} // namespace

// grid of one-wave workgroups; LDS: the fused drain's tile (kServeFusedMaxN
// bytes per row) plus the staging flag, or the ordered drain's tour
template <bool ORDERED, bool WIDE>
__device__ __forceinline__ void drain(ServeCtl ctl, ServeQueue *q)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const int lane = threadIdx.x;
    const long long start = ticks();
    long long idle_since = start;
    const int home = (int)(blockIdx.x & (kServeParts - 1));
    ClaimCache cc{0u, -1, 0, 1};
    JobView jv{};
    int slot, tile, count, part;
    bool fresh;
    while (claim(q, ctl.jobs, start, idle_since, ctl, lane, home, cc, slot, tile, count, part,
                 fresh)) {
        if (fresh) { // a job this wave has not run before: its descriptor
            jv = read_job(ctl.jobs + slot);
            if (ORDERED) { // and its tour's customer order for the gather
                uint16_t *cust = reinterpret_cast<uint16_t *>(lds);
                const int padded = (jv.n + 15) & ~15; // within the array: its length is
                                                      // max_len rounded up to 16
                for (int j = lane; j < padded; j += kWave)
                    cust[j] = j < jv.n ? (uint16_t)jv.tab[j + 1].x : (uint16_t)0;
                __syncthreads();
            }
        }
        TileAcc acc{0, 0, false, false};
        for (int i = 0; i < count; ++i)
            run_tile<ORDERED, WIDE>(ctl, jv, tile + i, lds, lane, acc);
        finish_chunk(ctl, jv, slot, part, count, acc, lane);
        idle_since = ticks();
    }
}

// one kernel per queue
__global__ __launch_bounds__(kWave) void serve_drain_fused32(ServeCtl ctl, ServeQueue *q)
{
    drain<false, false>(ctl, q);
}
__global__ __launch_bounds__(kWave) void serve_drain_fused64(ServeCtl ctl, ServeQueue *q)
{
    drain<false, true>(ctl, q);
}
__global__ __launch_bounds__(kWave) void serve_drain_ordered32(ServeCtl ctl, ServeQueue *q)
{
    drain<true, false>(ctl, q);
}
__global__ __launch_bounds__(kWave) void serve_drain_ordered64(ServeCtl ctl, ServeQueue *q)
{
    drain<true, true>(ctl, q);
}

// one workgroup per admitted job: its tables (tab, ab, rec, as laid out in
// its arena block, which tab starts) and then its descriptor, both from the
// job's pinned staging area (descriptor first, tables after it)
constexpr int kAdmitThreads = 256;

__global__ __launch_bounds__(kAdmitThreads) void serve_admit_kernel(ServeJob *jobs,
                                                                    const char *stage_base,
                                                                    size_t stage_bytes,
                                                                    AdmitBatch batch)
{
    const int s = batch.slot[blockIdx.x];
    const char *st = stage_base + (size_t)s * stage_bytes;
    const ServeJob *src = reinterpret_cast<const ServeJob *>(st);
    const int hb = src->head_bytes;
    uint8_t *dst = reinterpret_cast<uint8_t *>(const_cast<int2 *>(src->tab));
    const uint8_t *from = reinterpret_cast<const uint8_t *>(st) + kStageHead;
    for (int w = threadIdx.x; w < hb / 16; w += kAdmitThreads)
        reinterpret_cast<u32x4 *>(dst)[w] = reinterpret_cast<const u32x4 *>(from)[w];
    for (int b = (hb & ~15) + threadIdx.x; b < hb; b += kAdmitThreads)
        dst[b] = from[b];
    constexpr int words = (int)(sizeof(ServeJob) / sizeof(uint32_t));
    const uint32_t *js = reinterpret_cast<const uint32_t *>(src);
    uint32_t *jd = reinterpret_cast<uint32_t *>(jobs + s);
    for (int w = threadIdx.x; w < words; w += kAdmitThreads)
        jd[w] = js[w];
}

// one wave: the batch's slots appended to their queues, the new tails
// published with release order (the jobs' descriptors and tables were
// written by the launches before it on the same stream)
__global__ __launch_bounds__(kWave) void serve_publish_kernel(ServeQueues queues,
                                                              PublishBatch batch)
{
    if (threadIdx.x == 0) {
        uint32_t t[kServeQueues], b[kServeQueues];
        for (int k = 0; k < kServeQueues; ++k)
            b[k] = t[k] = __hip_atomic_load(&queues.q[k]->tail, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        for (int i = 0; i < batch.count; ++i) {
            const int s = batch.entry[i] & ((1 << 28) - 1);
            const int k = (batch.entry[i] >> 28) & (kServeQueues - 1);
            __hip_atomic_store(&queues.q[k]->ring[t[k]++ & (kServeQueueCap - 1)], s,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        for (int k = 0; k < kServeQueues; ++k)
            if (t[k] != b[k])
                __hip_atomic_store(&queues.q[k]->tail, t[k], __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

// LDS of a drain wave: the fused drain's tile (kServeFusedMaxN bytes per
// row) and staging flag; the ordered drain's tour (u16 per position, the
// length rounded up to 16), its staged rows (kServeStageRows x
// kServeStageMaxN bytes) and staging flag
static size_t drain_lds(bool ordered, int32_t max_len)
{
    return ordered ? 2 * (((size_t)max_len + 15) & ~(size_t)15) +
                         (size_t)kServeStageRows * kServeStageMaxN + 16
                   : (((size_t)kWave * kServeFusedMaxN + 15) & ~(size_t)15) + 16;
}

typedef void (*DrainKernel)(ServeCtl, ServeQueue *);

static DrainKernel drain_kernel(int queue)
{
    switch (queue) {
    case 0: return serve_drain_fused32;
    case 1: return serve_drain_fused64;
    case 2: return serve_drain_ordered32;
    default: return serve_drain_ordered64;
    }
}

static const void *drain_fn(int queue) { return reinterpret_cast<const void *>(drain_kernel(queue)); }

int serve_drain_grid(int queue, int32_t max_len)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const bool ordered = serve_queue_ordered(queue);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, drain_fn(queue), kWave,
                                                     drain_lds(ordered, max_len)) != hipSuccess ||
        per < 1)
        per = 1;
    // leave one workgroup slot per CU (and the LDS and registers it needs)
    // to the admission launches, so a round is not held up until drain
    // waves retire; one drain may otherwise fill the device
    if (per >= 2)
        per -= 1;
    return cus * per;
}

hipError_t serve_launch_drain(int queue, const ServeCtl &ctl, ServeQueue *q, int grid,
                              hipStream_t stream)
{
    const size_t lds = drain_lds(serve_queue_ordered(queue), ctl.max_len);
    hipLaunchKernelGGL(drain_kernel(queue), dim3(grid), dim3(kWave), lds, stream, ctl, q);
    return hipGetLastError();
}

hipError_t serve_launch_admit(ServeJob *jobs, const char *stage_base, size_t stage_bytes,
                              const AdmitBatch &batch, hipStream_t stream)
{
    hipLaunchKernelGGL(serve_admit_kernel, dim3(batch.count), dim3(kAdmitThreads), 0, stream,
                       jobs, stage_base, stage_bytes, batch);
    return hipGetLastError();
}

hipError_t serve_launch_publish(const ServeQueues &queues, const PublishBatch &batch,
                                hipStream_t stream)
{
    hipLaunchKernelGGL(serve_publish_kernel, dim3(1), dim3(kWave), 0, stream, queues, batch);
    return hipGetLastError();
}

} // namespace splitk
