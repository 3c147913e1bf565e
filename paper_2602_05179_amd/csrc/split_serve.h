// split_serve.h -- device-visible structures of the served form (the job
// table, the work queue and the host-visible results), shared by the drain
// kernels (split_serve.hip) and the scheduler (split_server.cpp).  Not part
// of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace splitk {

constexpr int kServeQueueCap = 1 << 14;  // ring entries per queue (power of two)
constexpr int kServeMaxJobs = 4096;      // job-table slots
constexpr int kServeScratchSlots = 16;   // exact-fallback value histories
constexpr int kServeFusedMaxN = 256;     // pools staged whole in LDS by the fused drain
constexpr int kServeStageMaxN = 1024;    // pools the ordered drain stages in LDS by row batches
constexpr int kServeStageRows = 8;       // rows per batch (a multiple of 8: batches start 16-byte aligned)

// Window variants a served job can take (chosen by capacity on the host).
enum ServeVariant : int32_t { SV_R32_6 = 0, SV_R32_8 = 1, SV_R64_16 = 2 };

// Work queues: (demand path) x (ring width).  A drain kernel serves one
// queue, so the 32-slot drains are not held to the register budget of the
// 64-slot ring and run more waves per SIMD.
constexpr int kServeQueues = 4;
__host__ __device__ inline int serve_queue(bool ordered, int32_t variant)
{
    return (ordered ? 2 : 0) + (variant == SV_R64_16 ? 1 : 0);
}
__host__ __device__ inline bool serve_queue_ordered(int q) { return q >= 2; }
__host__ __device__ inline bool serve_queue_wide(int q) { return (q & 1) != 0; }

// Tile claims and completion counts of a job are spread over kServeParts
// partitions of its tiles (partition p holds tiles [tiles*p/P, tiles*(p+1)/P)),
// each counter in its own 128-byte line: every drain wave starts claiming
// from the partition its workgroup index selects, so the device-scope
// atomics of concurrent waves fall on different lines instead of queueing
// on one.
constexpr int kServeParts = 8;
constexpr int kServeChunkMax = 8;

struct alignas(128) ServePart {
    int32_t next;   // tiles of the partition claimed
    int32_t done;   // tiles of the partition finished
    long long sum;  // exact sum of the partition's finite costs
    long long ninf; // number of its SPLIT_INF costs
};

// One admitted request.  The host fills every field (device counters zero,
// parts_done = the number of empty partitions); drain waves read it after
// claiming one of its tiles.
struct alignas(128) ServeJob {
    const int16_t *demands; // [S][N] scenario-major
    const uint8_t *perm;    // ordered path: [S][pitch] tour-ordered bytes, written by the
                            // drain wave that runs each tile (else null)
    const int2 *tab;        // [n + kTabPad] {customer index, c_j}, entry 0 and pads zero
    const int2 *ab;         // [n] {a_j, b_j}
    int32_t *costs;         // [S] per-scenario V(n) or SPLIT_INF
    int64_t S;
    int32_t N, n, Q, f0, bn, tiles, variant, pitch, seq;
    int32_t head_bytes; // bytes of tab, ab and rec (staged after the descriptor)
    int32_t chunk;      // tiles a wave claims at once (1..kServeChunkMax)
    // device counters
    int32_t parts_done; // partitions finished (starts at the number of empty ones)
    int32_t flags;      // 1 negative demand, 2 no fallback scratch in time
    ServePart part[kServeParts];
};

__host__ __device__ inline int32_t serve_part_lo(int32_t tiles, int p)
{
    return (int32_t)((int64_t)tiles * p / kServeParts);
}

// Result of a job slot, written by the wave that finishes the job's last
// tile into host-visible pinned memory (seq last, with release order).
struct ServeResult {
    long long sum;
    double mean;
    int32_t flags;
    int32_t seq;
};

// A work queue: job slots in publication order; waves take tiles from the
// job at `head` and advance it once that job has no tiles left.
struct ServeQueue {
    uint32_t head, tail, pad[62];
    int32_t ring[kServeQueueCap];
};

// Everything a drain wave needs besides its queue.
struct ServeCtl {
    ServeJob *jobs;          // [kServeMaxJobs] device
    ServeResult *results;    // [kServeMaxJobs] host-visible pinned
    int *scratch;            // [kServeScratchSlots][64 * (max_len + 1)]
    uint32_t *scratch_mask;  // busy bits of the scratch slots
    int32_t max_len;
    int32_t pad;
    long long idle_ticks;    // wall-clock ticks (100 MHz) a wave waits on an empty queue
    long long life_ticks;    // wall-clock ticks after which a wave takes no new tile
};

// launchers (split_serve.hip)
hipError_t serve_launch_drain(int queue, const ServeCtl &ctl, ServeQueue *q, int grid,
                              hipStream_t stream);
int serve_drain_grid(int queue, int32_t max_len); // workgroups that fill the device
// One admission round, two launches on the scheduler's copy stream:
//   admit   -- one workgroup per job: its tables (tab, ab, rec) from its
//              pinned staging area into its arena block, its descriptor into
//              the job table (each slot's staging area holds the descriptor,
//              then the tables as laid out in the arena block);
//   publish -- one wave: the slots appended to their queues (entry = slot |
//              queue << 28), new tails published with release order.
constexpr int kPublishMax = 255;
constexpr size_t kStageHead = (sizeof(ServeJob) + 255) & ~(size_t)255; // tables start here
struct AdmitBatch {
    int32_t count;
    int32_t slot[kPublishMax];
};
struct PublishBatch {
    int32_t count;
    int32_t entry[kPublishMax];
};
hipError_t serve_launch_admit(ServeJob *jobs, const char *stage_base, size_t stage_bytes,
                              const AdmitBatch &batch, hipStream_t stream);
struct ServeQueues {
    ServeQueue *q[kServeQueues];
};
hipError_t serve_launch_publish(const ServeQueues &queues, const PublishBatch &batch,
                                hipStream_t stream);

} // namespace splitk
