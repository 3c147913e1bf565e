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

// Window variants a served job can take (chosen by capacity on the host).
enum ServeVariant : int32_t { SV_R32_6 = 0, SV_R32_8 = 1, SV_R64_16 = 2 };

// One admitted request.  The host fills every field except the device
// counters (zero at publication); drain waves read it after claiming one
// of its tiles.
struct ServeJob {
    const int16_t *demands; // [S][N] scenario-major
    const uint8_t *perm;    // ordered path: [S][pitch] tour-ordered bytes (else null)
    const uint8_t *tile_bad; // ordered path: [tiles] tile needs the exact path (else null)
    const int2 *tab;        // [n + kTabPad] {customer index, c_j}, entry 0 and pads zero
    const int2 *ab;         // [n] {a_j, b_j}
    int32_t *costs;         // [S] per-scenario V(n) or SPLIT_INF
    int64_t S;
    int32_t N, n, Q, f0, bn, tiles, variant, pitch, seq, pad0;
    // device counters
    int32_t next_tile;  // tiles claimed
    int32_t tiles_done; // tiles finished
    int32_t flags;      // 1 negative demand, 2 no fallback scratch in time
    int32_t pad1;
    long long sum;      // exact sum of finite costs
    long long ninf;     // number of SPLIT_INF costs
};

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
hipError_t serve_launch_drain(bool ordered, const ServeCtl &ctl, ServeQueue *q, int grid,
                              hipStream_t stream);
int serve_drain_grid(bool ordered); // workgroups that fill the device
// A batch of admitted jobs to publish: entry = slot | (queue << 30); each
// slot's descriptor sits at the start of its pinned staging area.
struct PublishBatch {
    int32_t count;
    int32_t entry[255];
};
constexpr int kPublishMax = 255;
hipError_t serve_launch_publish(ServeQueue *q0, ServeQueue *q1, ServeJob *jobs,
                                const char *stage_base, size_t stage_bytes,
                                const PublishBatch &batch, hipStream_t stream);

} // namespace splitk
