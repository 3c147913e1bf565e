// split_internal.h -- types shared by the kernels and the host side of the
// library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "split_check.h"

namespace splitk {

// Per-tour constants produced by the prep kernel.
struct TourRec {
    int n;      // tour length
    int f0;     // first potential: V(0) + a_1 = c[0][sigma_1]
    int bn;     // b_n = D_n + c[sigma_n][0]; V(n) = m_n + b_n
    int status; // 0 ok, else a bit set of validation failures
    int maxc;   // largest travel cost on the tour's route legs
};

// Device scratch carved from one caller- or library-owned allocation.
struct Workspace {
    int2 *tab;             // [T * (max_len + kTabPad)] {customer index, c_j}, padded
    int2 *ab;              // [T * max_len] {a_j, b_j} (exact fallback)
    TourRec *rec;          // [T]
    long long *slots;      // [T * slots_per_tour(T) * kSlotStride] per-tour {sum, #inf}
    int *list;             // [units] units handed to the exact fallback
    int *list_count;       // [1]
    int *done;             // [1] fallback blocks finished
    int *vscratch;         // [fallback blocks * 64 * (max_len + 1)] value history
    uint8_t *tile_bad;     // [tiles] ordered path: tile needs the exact fallback (or null)
    uint8_t *perm;         // [T * S * pitch] ordered path: demands in tour order (or null)
    int *order;            // [T] tour indices by decreasing length (batched fused path)
    int max_len;
};

// How the main kernel runs (one instantiation per compiled window variant).
struct Schedule {
    int ring;  // register ring length R (32 or 64)
    int first; // cells of the first head group (its check is issued one position early)
    int group; // cells of each later head group (0 = none)
    int every; // tail cells between exits on an empty EXEC
    int waves; // tours (waves) per workgroup sharing one staged tile; 0 = automatic
    int path;  // 0 = automatic, 1 = fused (tile staged in LDS), 2 = ordered (permute + stream)
};

// Optional events bracketing the main kernel launch (measurement only).
struct LaunchEvents {
    hipEvent_t before = nullptr;
    hipEvent_t after = nullptr;
};

constexpr int kTile = 64;            // scenarios per unit (one wave)
constexpr int kTabPad = 4;           // table entries besides positions 1..n: index 0, n+1..n+3
constexpr int kSlots = 64;           // partial-sum slots of a single tour (fewer when T > 1)
constexpr int kSlotStride = 16;      // int64 words between slots (128 bytes)
constexpr int kMaxLen = 65535;       // longest tour the library accepts
constexpr int kLdsLimit = 160 * 1024; // LDS bytes one workgroup may use on gfx950
constexpr int kFallbackBlocks = 64;  // waves of an exact-fallback launch (sizes the V scratch)

int64_t num_tiles(int64_t S);
size_t workspace_bytes(int32_t T, int32_t max_len, int32_t N, int64_t S, bool ordered);
Workspace carve_workspace(void *base, int32_t T, int32_t max_len, int32_t N, int64_t S,
                          bool ordered);
int waves_per_group(int32_t T, int32_t N);
bool ordered_path_possible(int32_t N, int32_t max_len);
bool use_ordered_path(int32_t T, int32_t N, int32_t max_len);
int32_t ordered_pitch(int32_t max_len); // row stride of the tour-ordered copy

// Writes the tour-ordered copy of every tile (ws.perm, ws.tile_bad).
hipError_t launch_permute(const int16_t *demands, int32_t N, int64_t S, int32_t T,
                          int32_t max_len, const Workspace &ws, hipStream_t stream);

// Per-tour tables, validation and accumulator reset for T tours (lens ==
// nullptr: one tour of length max_len).
hipError_t launch_prep(const int32_t *tours, const int32_t *lens, int32_t T, int32_t max_len,
                       const int32_t *dist, int32_t N, const Workspace &ws, hipStream_t stream);

hipError_t launch_eval(const int32_t *tours, const int32_t *lens, int32_t T, int32_t max_len,
                       const int32_t *dist, int32_t N, const int16_t *demands, int64_t S,
                       int32_t Q, int32_t *costs, int64_t *sums, double *means,
                       const Workspace &ws, hipStream_t stream, const Schedule &sched,
                       const LaunchEvents *ev = nullptr);

hipError_t launch_count_cells(const int32_t *tours, const int32_t *lens, int32_t T, int32_t N,
                              const int16_t *demands, int64_t S, int32_t Q, int64_t *cells,
                              hipStream_t stream);

Schedule default_schedule(int32_t N, int64_t S, int32_t Q);

// Schedule for a call (override > tuned entry > default) and its path.
Schedule choose_schedule(int32_t T, int32_t max_len, int32_t N, int64_t S, int32_t Q,
                         bool *ordered);

bool schedule_supported(const Schedule &s);

hipError_t launch_count_mismatch(const int32_t *a, const int32_t *b, int64_t n, int64_t *out,
                                 hipStream_t stream);

// Every compiled (ring, first, group, every) window variant, in a fixed order.
int compiled_schedules(Schedule *out, int cap);

// Route recovery (one giant tour over S scenarios).
struct RouteVariant {
    int ring;  // register ring length R (32 or 64)
    int first; // cells of the first head group (its check is issued one position early)
    int group; // cells of each later head group (0 = none)
    int every; // tail cells between exits on an empty EXEC
};
bool route_variant_supported(const RouteVariant &v);
int compiled_route_variants(RouteVariant *out, int cap);
RouteVariant choose_route_variant(int32_t Q); // override, else the default for Q
void set_route_override(const RouteVariant &v); // ring 0 = automatic
// whether a call streams the tour-ordered copy (path override, else by
// the demand bytes per wave of the LDS tile); the workspace holds the copy then
bool routes_ordered(int32_t n, int32_t N);
void set_route_path(int path); // 0 automatic, 1 LDS tile, 2 tour-ordered copy
size_t routes_workspace_bytes(int32_t n, int32_t N, int64_t S);
// where a route-recovery workspace keeps the position table of a gathered tile
int2 *routes_position_table(void *workspace, int32_t n, int32_t N, int64_t S);
hipError_t launch_routes(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                         const int16_t *demands, int64_t S, int32_t Q, int32_t *costs,
                         uint16_t *pred, uint16_t *cuts, int32_t *nroutes, const Workspace &ws,
                         int2 *tabp, hipStream_t stream, const RouteVariant &v,
                         const LaunchEvents *ev = nullptr);

// Shape bucket used by the tuning table.
struct TuneKey {
    int tours, len, pool, scen, cap;
    bool operator<(const TuneKey &o) const;
};
TuneKey tune_key(int32_t T, int32_t max_len, int32_t N, int64_t S, int32_t Q);
// Tuned schedule for this shape if one was recorded (split_tune_device / load).
bool tuned_schedule(const TuneKey &k, Schedule *out);

} // namespace splitk
