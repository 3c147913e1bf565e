// split_device.h -- device-side helpers shared by the evaluation and the
// route-recovery kernels (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "split_internal.h"

namespace splitk {

constexpr int kWave = 64;
constexpr int kInf = 1 << 30;    // "+inf" potential sentinel
constexpr int kNeg = -(1 << 30); // threshold of ring slots before the tour start

enum : int { ST_OK = 0, ST_BAD_TOUR = 1, ST_BAD_DEMAND = 2 };

typedef const __attribute__((address_space(4))) int CInt; // scalar-loadable table words
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Global-memory views of generic pointers: loads through them are global
// (not flat) loads, counted by vmcnt only, so a prefetch in flight is not
// waited for by the lgkmcnt waits of scalar and LDS loads, and the compiler
// can wait for one load without draining the younger ones.  Use only for
// pointers into device memory.
typedef const __attribute__((address_space(1))) u32x4 GU32x4;
typedef const __attribute__((address_space(1))) int16_t GI16;

// table entry j of a per-tour table viewed as scalar-loadable words
__device__ __forceinline__ int2 tab_at(CInt *tab, int j) { return make_int2(tab[2 * j], tab[2 * j + 1]); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ long long wave_sum_i64(long long v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ int wave_sum_i32(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, kWave);
    return v;
}

// ---------------------------------------------------------------------------
// tile staging: int16 rows [rows x N] (contiguous) -> LDS bytes [rows x N]
// returns false (uniformly) when some value is outside [0, 255]
// s_bad: an LDS word outside the staged bytes (the block-wide "bad" flag)
//
// The 16-byte chunks of a thread are fetched BATCH at a time, all in
// flight together before any is narrowed: with 16 a one-wave block stages
// a 64 x 200 tile (25 chunks per lane) in two memory round trips instead of
// one per four chunks, with 28 in one.  The ring registers of the recursion
// are not live yet, so a batch costs occupancy only where its registers
// exceed the recursion's (the main tile kernel: 142-152 VGPRs at 28, still
// three waves per SIMD, its LDS limit).
// ---------------------------------------------------------------------------
constexpr int kStageBatch = 16;

__device__ __forceinline__ uint2 narrow_chunk(const u32x4 v, uint32_t &bad)
{
    const uint32_t x0 = v.x, x1 = v.y, x2 = v.z, x3 = v.w;
    bad |= (x0 | x1 | x2 | x3) & 0xFF00FF00u;
    uint2 o;
    o.x = __builtin_amdgcn_perm(x1, x0, 0x06040200u);
    o.y = __builtin_amdgcn_perm(x3, x2, 0x06040200u);
    return o;
}

template <int BATCH = kStageBatch>
__device__ __forceinline__ bool stage_tile_u8(const int16_t *__restrict__ src, uint8_t *lds,
                                              int64_t elems, int tid, int nthreads, int &s_bad)
{
    if (tid == 0)
        s_bad = 0;
    __syncthreads();
    const int64_t chunks = elems >> 3; // full 8-element (16-byte) chunks
    uint32_t bad = 0;
    GU32x4 *src4 = (GU32x4 *)reinterpret_cast<const u32x4 *>(src);
    GI16 *gsrc = (GI16 *)src;
    uint2 *dst8 = reinterpret_cast<uint2 *>(lds);
    for (int64_t i = tid; i < chunks; i += (int64_t)BATCH * nthreads) {
        u32x4 v[BATCH];
#pragma unroll
        for (int r = 0; r < BATCH; ++r)
            if (i + (int64_t)r * nthreads < chunks)
                v[r] = __builtin_nontemporal_load(&src4[i + (int64_t)r * nthreads]);
#pragma unroll
        for (int r = 0; r < BATCH; ++r)
            if (i + (int64_t)r * nthreads < chunks)
                dst8[i + (int64_t)r * nthreads] = narrow_chunk(v[r], bad);
    }
    for (int64_t e = (chunks << 3) + tid; e < elems; e += nthreads) {
        const int v = gsrc[e];
        bad |= (v < 0 || v > 255) ? 1u : 0u;
        lds[e] = (uint8_t)v;
    }
    if (ballot(bad != 0) != 0 && (tid & (kWave - 1)) == 0)
        atomicOr(&s_bad, 1);
    __syncthreads();
    return s_bad == 0;
}

// ---------------------------------------------------------------------------
// gathered staging: the demands of one tour's positions, in tour order,
// lds[r * pitch + k] = demands[r * N + cust_k] as a byte for k < n, zero for
// n <= k < pitch (cust_k = tab[k + 1].x, the per-tour table's customer
// index).  Lanes take consecutive positions of one scenario row at a time,
// so each load instruction reads a few lines of that row.  Returns false
// (uniformly) when some value is outside [0, 255].
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool stage_tile_gather_u8(const int16_t *__restrict__ src, int N,
                                                     int rows, const int2 *__restrict__ tab,
                                                     int n, int pitch, uint8_t *lds, int tid,
                                                     int nthreads, int &s_bad)
{
    if (tid == 0)
        s_bad = 0;
    __syncthreads();
    uint32_t bad = 0;
    for (int k0 = 0; k0 < pitch; k0 += nthreads) {
        const int k = k0 + tid;
        const int cust = k < n ? tab[k + 1].x : -1;
        int r = 0;
        for (; r + 8 <= rows; r += 8) {
            int v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = cust >= 0 ? src[(int64_t)(r + u) * N + cust] : 0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                bad |= (v[u] < 0 || v[u] > 255) ? 1u : 0u;
                if (k < pitch)
                    lds[(r + u) * pitch + k] = (uint8_t)v[u];
            }
        }
        for (; r < rows; ++r) {
            const int v = cust >= 0 ? src[(int64_t)r * N + cust] : 0;
            bad |= (v < 0 || v > 255) ? 1u : 0u;
            if (k < pitch)
                lds[r * pitch + k] = (uint8_t)v;
        }
    }
    if (ballot(bad != 0) != 0 && (tid & (kWave - 1)) == 0)
        atomicOr(&s_bad, 1);
    __syncthreads();
    return s_bad == 0;
}

// ---------------------------------------------------------------------------
// Demand bytes of one lane's scenario, read in tour order by a recursion:
// position j's demand at position j - 2 (two ahead), after `init` has read
// positions 1 and 2.  ahead<U>(t) is called at position j = j0 + U of a
// block (j0 a multiple of 32), with t the table entry of position j + 2.

// a row in LDS, indexed through the table (the customer index for whole
// rows, position - 1 for a gathered tile)
struct LdsRow {
    const uint8_t *row;
    __device__ __forceinline__ void init(int2 t0, int2 t1, int &q1, int &q2) const
    {
        q1 = row[t0.x];
        q2 = row[t1.x];
    }
    template <int U> __device__ __forceinline__ int ahead(int2 t) const { return row[t.x]; }
    // demand of position j (random access, outside the recursion)
    __device__ __forceinline__ int at(CInt *tab, int j) const { return row[tab_at(tab, j).x]; }
};

// the lane's row of the tour-ordered copy in global memory (byte j - 1 =
// position j, zero-padded to a multiple of 32 bytes plus 32), held 32 bytes
// at a time in registers with the next 32 in flight
struct StreamRow {
    const u32x4 *row;
    int segs; // 32-byte segments in the row (at least 2)
    int nseg; // segment held in nxt
    u32x4 cur[2], nxt[2];

    template <int B> __device__ __forceinline__ static int byte_of(const u32x4 (&seg)[2])
    {
        const u32x4 &v = seg[B >> 4];
        constexpr int w = (B >> 2) & 3;
        const uint32_t x = w == 0 ? v.x : w == 1 ? v.y : w == 2 ? v.z : v.w;
        return (int)((x >> (8 * (B & 3))) & 0xFFu);
    }
    __device__ __forceinline__ void init(int2, int2, int &q1, int &q2)
    {
        cur[0] = __builtin_nontemporal_load(row);
        cur[1] = __builtin_nontemporal_load(row + 1);
        nxt[0] = __builtin_nontemporal_load(row + 2);
        nxt[1] = __builtin_nontemporal_load(row + 3);
        nseg = 1;
        q1 = byte_of<0>(cur);
        q2 = byte_of<1>(cur);
    }
    template <int U> __device__ __forceinline__ int ahead(int2)
    {
        constexpr int B = (U + 1) & 31; // byte j + 1 of the row
        const int v = byte_of<B>(cur);
        if (B == 31) { // next 32 positions: rotate and fetch the segment after
            cur[0] = nxt[0];
            cur[1] = nxt[1];
            if (++nseg < segs) {
                nxt[0] = __builtin_nontemporal_load(row + 2 * nseg);
                nxt[1] = __builtin_nontemporal_load(row + 2 * nseg + 1);
            }
        }
        return v;
    }
    // demand of position j (random access, outside the recursion)
    __device__ __forceinline__ int at(CInt *, int j) const
    {
        return reinterpret_cast<const uint8_t *>(row)[j - 1];
    }
};

namespace {

// The per-tour table re-indexed for a gathered tile: entry j = {j - 1, c_j}
// for j = 1..n (the demand of position j is byte j - 1 of the lane's row),
// and {n, 0} for entry 0 and the padding entries (byte n of a row is zero).
__global__ void position_table_kernel(const int2 *__restrict__ tab, int n, int2 *__restrict__ out)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n + kTabPad;
         j += gridDim.x * blockDim.x)
        out[j] = (j >= 1 && j <= n) ? make_int2(j - 1, tab[j].y) : make_int2(n, 0);
}

} // namespace

// Whether a one-tour kernel stages the tour's demands gathered (64 x (n+1)
// bytes) instead of whole rows (64 x N bytes): when whole rows do not fit
// the LDS limit, or the tour covers at most half of the pool.
inline bool gather_tile(int32_t n, int32_t N, int lds_limit)
{
    const size_t rows_bytes = (((size_t)kWave * (size_t)N + 15) & ~(size_t)15) + 16;
    return rows_bytes > (size_t)lds_limit || 2 * ((int64_t)n + 1) <= (int64_t)N;
}

} // namespace splitk
