// split_kernels.hip -- gfx950 kernels of the scenario-batched split evaluator.
//
// The recursion (paper Sec. 2.3): V(0) = 0,
//   V(i) = min over admissible p < i of V(p) + W(p,i),
// with W(p,i) the cost of the route depot -> sigma_{p+1} .. sigma_i -> depot
// and "admissible" meaning the route's load is at most Q.
//
// Potential form used on the GPU.  With out_k = c[0][sigma_k],
// in_k = c[sigma_k][0], arc_k = c[sigma_k][sigma_{k+1}] and
// D_k = sum_{m<k} arc_m, the route cost splits into two one-index terms,
//   W(p,i) = a_{p+1} + b_i,   a_k = out_k - D_k,   b_i = D_i + in_i,
// so V(i) = b_i + min_{p in window(i)} f_p with f_p = V(p) + a_{p+1}.
// Writing m_i = min_{p in window(i)} f_p, the next potential is
//   f_i = m_i + c_i,   c_i = b_i + a_{i+1} = in_i + out_{i+1} - arc_i,
// and V(n) = m_n + b_n.  The window of admissible predecessors is a
// contiguous range [p_min(i), i-1] because demands are non-negative, and
// both of its ends are non-decreasing in i (the monotone structure the
// paper's deque kernel relies on, App. A "Pseudo-code for 2D kernel").
//
// Lane layout: one scenario per lane, a tile of 64 scenarios per wave.  A
// tile's demand rows (int16, scenario-major, contiguous in HBM) are streamed
// into LDS with 16-byte coalesced loads and narrowed to bytes when every
// value of the tile fits (the common case); each lane then gathers its
// demands through the tour from its own LDS row.  The per-position table
// {customer, c_i} is uniform across the wave and is read with scalar loads.
// The last R potentials f_p and thresholds L_p + Q of a lane live in
// registers; the position loop is unrolled R times so every ring slot is a
// compile-time register, and the masked window minimum of a position is the
// inline-assembly block of window_min_asm.inc (see gen_window_asm.py).
// A lane whose window reaches past the ring, and any tile whose demands do
// not fit a byte, are recomputed by an exact fallback kernel.
//
// Infeasible scenarios (some demand > Q) need no special case: an empty
// window leaves m = INF, and every later value stays >= INF because all
// route costs are non-negative, while feasible values stay < 2^29 under the
// documented cost guard; V(n) >= INF is reported as SPLIT_INF.
//
// Per-tour sums: every unit adds its exact int64 partial sum into one of
// kSlots per-tour slots (128 bytes apart, so concurrent atomics spread over
// L2 channels); the last block of the fallback kernel folds the slots into
// the tour's sum and mean (sum / S, one IEEE double division).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "split_eval.h"
#include "split_device.h"
#include "split_dp.h"
#include "split_internal.h"

namespace splitk {

// Partial-sum slots per tour: enough that no slot sees many atomics (a
// tour has ceil(S/64) units), few enough that the final fold stays short.
__host__ __device__ __forceinline__ int slots_per_tour(int32_t T)
{
    return T >= kSlots ? 1 : kSlots / (1 << (31 - __builtin_clz((unsigned)T)));
}

// slot k of tour t: {sum, number of SPLIT_INF costs}
__device__ __forceinline__ long long *slot_ptr(const Workspace &ws, int T, int t, int k)
{
    return ws.slots + ((int64_t)t * slots_per_tour(T) + k) * kSlotStride;
}

__device__ __forceinline__ void add_unit_result(const Workspace &ws, int T, int t, int64_t unit,
                                                long long sum, int ninf)
{
    long long *sp = slot_ptr(ws, T, t, (int)(unit % slots_per_tour(T)));
    if (sum)
        atomicAdd(reinterpret_cast<unsigned long long *>(sp), (unsigned long long)sum);
    if (ninf)
        atomicAdd(reinterpret_cast<unsigned long long *>(sp + 1), (unsigned long long)ninf);
}

// ---------------------------------------------------------------------------
// prep: per-tour table, validation, accumulator reset
// grid = num_tours blocks of 256 threads
// tab[t * (max_len + kTabPad) + j] = {customer index of position j, c_j} for
// j = 1..n, zero at j = 0 and for the padding entries n+1..n+3.
// lens == nullptr: a single tour of length max_len.
// ---------------------------------------------------------------------------
constexpr int kPrepThreads = 256;

__global__ __launch_bounds__(kPrepThreads) void prep_kernel(
    const int32_t *__restrict__ tours, const int32_t *__restrict__ lens, int32_t num_tours,
    int32_t max_len, const int32_t *__restrict__ dist, int32_t N, Workspace ws)
{
    __shared__ long long s_red[kPrepThreads / kWave];
    __shared__ int s_redi[kPrepThreads / kWave];
    __shared__ long long s_carry;
    __shared__ long long s_scan[kPrepThreads / kWave];

    const int t = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wid = tid / kWave;
    const int64_t N1 = (int64_t)N + 1;

    if (t == 0 && tid == 0) {
        *ws.list_count = 0;
        *ws.done = 0;
    }
    const int spt = slots_per_tour(num_tours);
    for (int i = tid; i < spt * kSlotStride; i += kPrepThreads)
        ws.slots[(int64_t)t * spt * kSlotStride + i] = 0;

    // offset of this tour in the concatenated array; an invalid earlier
    // length makes the layout ambiguous, so this tour is rejected too
    long long off = 0;
    int prev_bad = 0;
    for (int i = tid; i < t; i += kPrepThreads) {
        const int li = lens ? lens[i] : max_len;
        prev_bad |= (li < 0 || li > max_len) ? 1 : 0;
        off += li;
    }
    off = wave_sum_i64(off);
    prev_bad = wave_sum_i32(prev_bad);
    if (lane == 0) {
        s_red[wid] = off;
        s_redi[wid] = prev_bad;
    }
    __syncthreads();
    off = 0;
    prev_bad = 0;
#pragma unroll
    for (int w = 0; w < kPrepThreads / kWave; ++w) {
        off += s_red[w];
        prev_bad += s_redi[w];
    }
    __syncthreads();

    const int n = lens ? lens[t] : max_len;
    int bad = (n < 0 || n > max_len || prev_bad) ? 1 : 0;
    const int nn = bad ? 0 : n;
    int maxc = 0;
    if (tid == 0)
        s_carry = 0;
    __syncthreads();

    int2 *tab = ws.tab + (int64_t)t * (max_len + kTabPad);
    int2 *ab = ws.ab + (int64_t)t * max_len;
    for (int i = tid; i < kTabPad; i += kPrepThreads)
        tab[i == 0 ? 0 : nn + i] = make_int2(0, 0);
    int first_out = 0;
    for (int base = 0; base < nn; base += kPrepThreads) {
        const int k = base + tid; // tour position k+1 (0-based k)
        long long arc = 0;
        int c = 0, out = 0, in = 0, cn = 0, outn = 0, a = 0;
        if (k < nn) {
            c = tours[off + k];
            if (c < 1 || c > N) {
                bad = 1;
                c = 1;
            }
            out = dist[c];
            in = dist[(int64_t)c * N1];
            if (k + 1 < nn) {
                cn = tours[off + k + 1];
                if (cn < 1 || cn > N) {
                    bad = 1;
                    cn = 1;
                }
                a = dist[(int64_t)c * N1 + cn];
                outn = dist[cn];
                arc = a;
            }
            if (out < 0 || in < 0 || a < 0 || out > SPLIT_MAX_COST || in > SPLIT_MAX_COST ||
                a > SPLIT_MAX_COST)
                bad = 1;
            maxc = max(maxc, max(out, max(in, a)));
            if (k == 0)
                first_out = out;
        }
        // exclusive prefix of arc over positions: D_{k+1} = sum_{m<k} arc_m
        long long incl = arc;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            long long y = __shfl_up(incl, o, kWave);
            if (lane >= o)
                incl += y;
        }
        if (lane == kWave - 1)
            s_scan[wid] = incl;
        __syncthreads();
        long long pre = s_carry;
        for (int w = 0; w < wid; ++w)
            pre += s_scan[w];
        const long long Dk = pre + incl - arc;
        __syncthreads();
        if (tid == kPrepThreads - 1)
            s_carry = pre + incl;
        if (k < nn) {
            const long long ak = (long long)out - Dk;
            const long long bk = Dk + in;
            const int ck = (k + 1 < nn) ? (in + outn - (int)arc) : 0;
            tab[k + 1] = make_int2(c - 1, ck);
            ab[k] = make_int2((int)ak, (int)bk);
        }
        __syncthreads();
    }

    // reduce bad flag, largest cost and the first depot leg
    int b = bad, mc = maxc, fo = first_out;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        b |= __shfl_xor(b, o, kWave);
        mc = max(mc, __shfl_xor(mc, o, kWave));
        fo = max(fo, __shfl_xor(fo, o, kWave));
    }
    if (lane == 0)
        s_redi[wid] = b ? -1 : mc;
    if (tid == 0)
        s_red[0] = fo; // only thread 0 (position 1) holds a non-zero first leg
    __syncthreads();
    if (tid == 0) {
        int allbad = 0, allmax = 0;
        for (int w = 0; w < kPrepThreads / kWave; ++w) {
            if (s_redi[w] < 0)
                allbad = 1;
            else
                allmax = max(allmax, s_redi[w]);
        }
        // exactness guard: 3 * n * max cost < 2^29
        if ((long long)3 * nn * allmax >= (1LL << 29))
            allbad = 1;
        TourRec r;
        r.n = nn;
        r.f0 = (int)s_red[0]; // a_1 = c[0][sigma_1] since D_1 = 0
        r.bn = nn > 0 ? ab[nn - 1].y : 0;
        r.status = allbad ? ST_BAD_TOUR : ST_OK;
        r.maxc = allmax;
        ws.rec[t] = r;
    }
}

// ---------------------------------------------------------------------------
// main evaluation kernel: a workgroup of W waves stages one tile of 64
// scenario rows and runs W different tours over it (wave w takes tour
// g*W + w), so tours sharing a scenario set share one LDS copy of it.
// Workgroup b -> tile k = b / NG, tour group g = b % NG with NG = ceil(T/W):
// all tours of a tile run close together in time, so a shared demand tile
// is read from HBM about once per XCD.  The (tile, tour) unit id used by
// the fallback list is u = k*T + t.
// LDS: 64 x N demand bytes
// ---------------------------------------------------------------------------
constexpr int kMaxWavesPerGroup = 8;
// 16-byte chunks per thread in flight while a one-wave workgroup stages its
// tile: a 64 x 224 tile in one memory round trip (n = N = 200, S = 10^6,
// Q = 150: 253 -> 245 us against batches of 16).  Its registers (142-152
// VGPRs) allow three waves per SIMD, so it is used only where the tile's
// LDS already allows no more; multi-wave workgroups keep kStageBatch.
constexpr int kTileStageBatch = 28;

template <int R, int F, int G, int E, int SB>
__global__ __launch_bounds__(kWave *kMaxWavesPerGroup) void split_tile_kernel(
    const int16_t *__restrict__ demands, int32_t N, int64_t S, int32_t Q, int32_t T,
    int32_t *__restrict__ costs, Workspace ws, int32_t use_lds, int32_t by_length)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const int W = blockDim.x / kWave;
    const int NG = (T + W - 1) / W;
    const int64_t b = blockIdx.x;
    // by_length: tours taken in decreasing length (groups of similar
    // length finish together), group-major so the longest work starts
    // first; otherwise tile-major, so the groups sharing a tile run close
    // together and the tile is read from HBM about once
    int64_t k;
    int g;
    if (by_length) {
        const int64_t tiles = (S + kWave - 1) / kWave;
        g = (int)(b / tiles);
        k = b - (int64_t)g * tiles;
    } else {
        k = b / NG;
        g = (int)(b - k * NG);
    }
    const int lane = threadIdx.x & (kWave - 1);
    // uniform within the wave; readfirstlane lets the compiler keep the
    // tour's scalars (length, table pointer) in SGPRs
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int slot = g * W + wave;
    const int t = by_length && slot < T ? __builtin_amdgcn_readfirstlane(ws.order[slot]) : slot;
    const int64_t s0 = k * kWave;
    const int rows = (int)min<int64_t>(kWave, S - s0);

    bool ok = false;
    if (use_lds) {
        int &s_bad = *reinterpret_cast<int *>(lds + (((size_t)kWave * N + 15) & ~(size_t)15));
        ok = stage_tile_u8<SB>(demands + s0 * N, lds, (int64_t)rows * N, threadIdx.x, blockDim.x,
                               s_bad);
        __syncthreads();
    }
    if (t >= T)
        return;
    const int64_t u = k * T + t;
    const TourRec rec = ws.rec[t];
    int32_t *out = costs + (int64_t)t * S + s0;
    if (rec.status != ST_OK || rec.n == 0) {
        if (lane < rows)
            out[lane] = rec.status != ST_OK ? SPLIT_INF : 0;
        return;
    }
    bool redo = true;
    if (ok) {
        CInt *tab = (CInt *)(ws.tab + (int64_t)t * (ws.max_len + kTabPad));
        bool ovf = false;
        int v = 0;
        if (lane < rows) {
            const int m = dp_lane<R, F, G, E>(lds + (int64_t)lane * N, tab, rec.n, rec.f0,
                                              Q, ovf);
            v = m + rec.bn;
        }
        redo = ballot(ovf) != 0;
        if (!redo) {
            const bool fin = lane < rows && v < kInf;
            const bool inf = lane < rows && v >= kInf;
            if (lane < rows)
                out[lane] = inf ? SPLIT_INF : v;
            const long long sm = wave_sum_i64(fin ? (long long)v : 0LL);
            const int ni = wave_sum_i32(inf ? 1 : 0);
            if (lane == 0)
                add_unit_result(ws, T, t, u, sm, ni);
        }
    }
    if (redo && lane == 0) {
        const int slot = atomicAdd(ws.list_count, 1);
        ws.list[slot] = (int)u;
    }
}

// ---------------------------------------------------------------------------
// ordered path (large customer pools): the demands of each tile are first
// written in tour order as bytes, perm[t][s][j-1] = q_s(sigma_j), rows
// padded to `pitch` bytes (a multiple of 32, padding zero); the recursion
// kernel then streams each lane's own row 32 positions at a time straight
// into registers, so it needs no LDS and its occupancy is register-bound.
// ---------------------------------------------------------------------------
constexpr int kPermThreads = 256;

// grid = tiles; LDS: 64 x N demand bytes + flag word + tour (u16 per position)
__global__ __launch_bounds__(kPermThreads) void permute_tile_kernel(
    const int16_t *__restrict__ demands, int32_t N, int64_t S, int32_t T, int32_t pitch,
    Workspace ws)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const int64_t k = blockIdx.x;
    const int64_t s0 = k * kWave;
    const int rows = (int)min<int64_t>(kWave, S - s0);
    const size_t rows_bytes = ((size_t)kWave * N + 15) & ~(size_t)15;
    int &s_bad = *reinterpret_cast<int *>(lds + rows_bytes);
    uint16_t *cust = reinterpret_cast<uint16_t *>(lds + rows_bytes + 16);
    const bool ok = stage_tile_u8(demands + s0 * N, lds, (int64_t)rows * N, threadIdx.x,
                                  blockDim.x, s_bad);
    if (!ok) {
        if (threadIdx.x == 0)
            ws.tile_bad[k] = 1;
        return; // uniform: every tour's unit of this tile takes the exact fallback
    }
    if (threadIdx.x == 0)
        ws.tile_bad[k] = 0;
    const int chunks = pitch / 16;
    for (int t = 0; t < T; ++t) {
        const TourRec rec = ws.rec[t];
        const int n = rec.status == ST_OK ? rec.n : 0;
        const int2 *tab = ws.tab + (int64_t)t * (ws.max_len + kTabPad);
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += blockDim.x)
            cust[j] = (uint16_t)tab[j + 1].x;
        __syncthreads();
        uint8_t *dst = ws.perm + ((int64_t)t * S + s0) * pitch;
        for (int idx = threadIdx.x; idx < rows * chunks; idx += blockDim.x) {
            const int r = idx / chunks;
            const int c = idx - r * chunks;
            const uint8_t *row = lds + (int64_t)r * N;
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t x = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int j = c * 16 + q * 4 + b;
                    const uint32_t v = j < n ? row[cust[j]] : 0u;
                    x |= v << (8 * b);
                }
                w[q] = x;
            }
            u32x4 o = {w[0], w[1], w[2], w[3]};
            __builtin_nontemporal_store(o, reinterpret_cast<u32x4 *>(dst + (int64_t)r * pitch) + c);
        }
    }
}

// grid = units (u -> tile u / T, tour u % T), one wave each
template <int R, int F, int G, int E>
__global__ __launch_bounds__(kWave) void split_ordered_kernel(int64_t S, int32_t Q, int32_t T,
                                                              int32_t pitch,
                                                              int32_t *__restrict__ costs,
                                                              Workspace ws)
{
    const int64_t u = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t k = u / T;
    const int t = (int)(u - k * T);
    const int64_t s0 = k * kWave;
    const int rows = (int)min<int64_t>(kWave, S - s0);
    const TourRec rec = ws.rec[t];
    int32_t *out = costs + (int64_t)t * S + s0;
    if (rec.status != ST_OK || rec.n == 0) {
        if (lane < rows)
            out[lane] = rec.status != ST_OK ? SPLIT_INF : 0;
        return;
    }
    bool redo = ws.tile_bad[k] != 0;
    if (!redo) {
        CInt *tab = (CInt *)(ws.tab + (int64_t)t * (ws.max_len + kTabPad));
        bool ovf = false;
        int v = 0;
        if (lane < rows) {
            const uint8_t *rowb = ws.perm + ((int64_t)t * S + s0 + lane) * pitch;
            const int m = dp_lane_ordered<R, F, G, E>(rowb, pitch, tab, rec.n, rec.f0, Q, ovf);
            v = m + rec.bn;
        }
        redo = ballot(ovf) != 0;
        if (!redo) {
            const bool fin = lane < rows && v < kInf;
            const bool inf = lane < rows && v >= kInf;
            if (lane < rows)
                out[lane] = inf ? SPLIT_INF : v;
            const long long sm = wave_sum_i64(fin ? (long long)v : 0LL);
            const int ni = wave_sum_i32(inf ? 1 : 0);
            if (lane == 0)
                add_unit_result(ws, T, t, u, sm, ni);
        }
    }
    if (redo && lane == 0) {
        const int slot = atomicAdd(ws.list_count, 1);
        ws.list[slot] = (int)u;
    }
}

// ---------------------------------------------------------------------------
// exact fallback for listed units (any window length, any demand value),
// straight from the definition with the value history in global scratch;
// the last block to finish folds every tour's slots into its sum and mean
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWave) void fallback_final_kernel(const int16_t *__restrict__ demands,
                                                               int32_t N, int64_t S, int32_t Q,
                                                               int32_t T, int32_t *costs,
                                                               int64_t *sums, double *means,
                                                               Workspace ws)
{
    const int lane = threadIdx.x;
    const int count = *ws.list_count;
    int *V = ws.vscratch + (int64_t)blockIdx.x * kWave * (ws.max_len + 1);
    for (int li = blockIdx.x; li < count; li += gridDim.x) {
        const int64_t u = ws.list[li];
        const int64_t k = u / T;
        const int t = (int)(u - k * T);
        const int64_t s0 = k * kWave;
        const int rows = (int)min<int64_t>(kWave, S - s0);
        const TourRec rec = ws.rec[t];
        const int2 *tab = ws.tab + (int64_t)t * (ws.max_len + kTabPad);
        const int2 *ab = ws.ab + (int64_t)t * ws.max_len;
        const int n = rec.n;
        int v = 0;
        bool negq = false;
        if (lane < rows)
            v = exact_lane(demands + (s0 + lane) * N, tab, ab, n, Q, V, lane, negq);
        if (ballot(negq) != 0) {
            if (lane == 0)
                atomicOr(&ws.rec[t].status, ST_BAD_DEMAND);
        }
        const bool fin = lane < rows && v < kInf;
        const bool inf = lane < rows && v >= kInf;
        if (lane < rows)
            costs[(int64_t)t * S + s0 + lane] = inf ? SPLIT_INF : v;
        const long long s = wave_sum_i64(fin ? (long long)v : 0LL);
        const int ni = wave_sum_i32(inf ? 1 : 0);
        if (lane == 0)
            add_unit_result(ws, T, t, u, s, ni);
    }

    // last block: per-tour exact sum over slots, mean = sum / S
    int last = 0;
    if (lane == 0) {
        __threadfence();
        last = atomicAdd(ws.done, 1) == (int)gridDim.x - 1;
    }
    last = __shfl(last, 0, kWave);
    if (!last)
        return;
    __threadfence();
    // lanes cover (tour, slot) pairs; slots of one tour sit in a group of
    // spt adjacent lanes (spt is a power of two dividing 64)
    const int spt = slots_per_tour(T);
    for (int base = 0; base < T * spt; base += kWave) { // uniform loop: every lane active
        const int idx = base + lane;
        const int t = idx / spt;
        const int kk = idx - t * spt;
        long long tot = 0, ninf = 0;
        int status = ST_OK;
        if (t < T) {
            long long *sp = slot_ptr(ws, T, t, kk);
            tot = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ninf = __hip_atomic_load(sp + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            status = __hip_atomic_load(&ws.rec[t].status, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
        for (int o = 1; o < spt; o <<= 1) {
            tot += __shfl_xor(tot, o, kWave);
            ninf += __shfl_xor(ninf, o, kWave);
        }
        if (t < T && kk == 0) {
            if (status != ST_OK) {
                sums[t] = SPLIT_SUM_INVALID;
                means[t] = __builtin_nan("");
            } else if (ninf) {
                sums[t] = INT64_MAX;
                means[t] = __builtin_inf();
            } else {
                sums[t] = tot;
                means[t] = (double)tot / (double)S;
            }
        }
        // invalid tours (rare): every cost of the tour becomes SPLIT_INF
        uint64_t bad = ballot(t < T && kk == 0 && status != ST_OK);
        while (bad) {
            const int l = __builtin_ctzll(bad);
            bad &= bad - 1;
            const int64_t tb = (base + l) / spt;
            for (int64_t i = lane; i < S; i += kWave)
                costs[tb * S + i] = SPLIT_INF;
        }
    }
}

// ---------------------------------------------------------------------------
// Bellman-cell counter: per lane, two running loads bracket the window
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWave) void count_cells_kernel(const int32_t *__restrict__ tours,
                                                            const int32_t *__restrict__ lens,
                                                            int32_t T, int32_t N,
                                                            const int16_t *__restrict__ demands,
                                                            int64_t S, int32_t Q,
                                                            unsigned long long *__restrict__ cells)
{
    const int lane = threadIdx.x;
    const int64_t u = blockIdx.x;
    const int64_t k = u / T;
    const int t = (int)(u - k * T);
    const int64_t s = k * kWave + lane;
    long long off = 0;
    for (int i = 0; i < t; ++i)
        off += lens[i];
    const int n = lens[t];
    const int32_t *tour = tours + off;
    long long cnt = 0;
    if (s < S) {
        const int16_t *qrow = demands + s * N;
        auto q_at = [&](int pos) { // demand of tour position pos (ids clamped into range)
            const int c = min(max(tour[pos - 1], 1), N);
            return (int)qrow[c - 1];
        };
        int L = 0, Ll = 0, l = 0; // window [l, j-1]; Ll = load of positions 1..l
        for (int j = 1; j <= n; ++j) {
            L += q_at(j);
            while (l < j && L - Ll > Q) {
                ++l;
                Ll += q_at(l);
            }
            cnt += j - l;
        }
    }
    cnt = wave_sum_i64(cnt);
    if (lane == 0)
        atomicAdd(&cells[t], (unsigned long long)cnt);
}

// ---------------------------------------------------------------------------
// tuner support: number of positions where two int32 arrays differ
// ---------------------------------------------------------------------------
__global__ void count_mismatch_kernel(const int32_t *__restrict__ a, const int32_t *__restrict__ b,
                                      int64_t n, unsigned long long *__restrict__ out)
{
    long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        c += a[i] != b[i];
    c = wave_sum_i64(c);
    if ((threadIdx.x & (kWave - 1)) == 0 && c)
        atomicAdd(out, (unsigned long long)c);
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
__global__ void zero_i64_kernel(int64_t *p, int32_t n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0;
}

int64_t num_tiles(int64_t S) { return (S + kTile - 1) / kTile; }

// order[r] = the tour of rank r by decreasing length (ties by index); an
// invalid length ranks as 0 (its waves return at once).  One block; the
// lengths are staged in LDS and the rank of a tour is a count over all
// tours, O(T^2 / threads) LDS reads per launch.
constexpr int kOrderThreads = 1024;
constexpr int32_t kOrderMaxTours = 4096;

__global__ __launch_bounds__(kOrderThreads) void order_kernel(const int32_t *__restrict__ lens,
                                                              int32_t T, int32_t max_len,
                                                              int *__restrict__ order)
{
    __shared__ int s_len[kOrderMaxTours];
    for (int i = threadIdx.x; i < T; i += kOrderThreads) {
        const int li = lens[i];
        s_len[i] = li < 0 || li > max_len ? 0 : li;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < T; i += kOrderThreads) {
        const int ni = s_len[i];
        int rank = 0;
        for (int j = 0; j < T; ++j) {
            const int nj = s_len[j]; // the same address across the wave: a broadcast
            rank += (nj > ni || (nj == ni && j < i)) ? 1 : 0;
        }
        order[rank] = i;
    }
}

hipError_t launch_prep(const int32_t *tours, const int32_t *lens, int32_t T, int32_t max_len,
                       const int32_t *dist, int32_t N, const Workspace &ws, hipStream_t stream)
{
    hipLaunchKernelGGL(prep_kernel, dim3(T), dim3(kPrepThreads), 0, stream, tours, lens, T,
                       max_len, dist, N, ws);
    return hipGetLastError();
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int32_t ordered_pitch(int32_t max_len) { return ((max_len + 31) / 32) * 32 + 32; }

// Tours per workgroup: enough to keep the shared tile's LDS per wave small.
int waves_per_group(int32_t T, int32_t N)
{
    const int64_t bytes = (int64_t)kTile * N;
    int W = 1;
    while (W < kMaxWavesPerGroup && W < T && bytes / W > 8 * 1024)
        W *= 2;
    return W < T ? W : T;
}

// LDS bytes the permute kernel needs: rows + flag + tour (u16 per position)
static size_t permute_lds_bytes(int32_t N, int32_t max_len)
{
    return (((size_t)kTile * (size_t)N + 15) & ~(size_t)15) + 16 + 2 * ((size_t)max_len + 1);
}

// Ordered path when a fused workgroup would need more than 16 KB of LDS per
// wave (large pools, few tours), as long as the permute tile fits in LDS.
bool ordered_path_possible(int32_t N, int32_t max_len)
{
    return permute_lds_bytes(N, max_len) <= (size_t)kLdsLimit && N < 65535;
}

bool use_ordered_path(int32_t T, int32_t N, int32_t max_len)
{
    const int W = waves_per_group(T, N);
    return (int64_t)kTile * N / W > 16 * 1024 && ordered_path_possible(N, max_len);
}

size_t workspace_bytes(int32_t T, int32_t max_len, int32_t N, int64_t S, bool ordered)
{
    (void)N;
    const size_t units = (size_t)T * (size_t)num_tiles(S);
    size_t b = 0;
    b += align256((size_t)T * ((size_t)max_len + kTabPad) * sizeof(int2));
    b += align256((size_t)T * max_len * sizeof(int2));
    b += align256((size_t)T * sizeof(TourRec));
    b += align256((size_t)T * slots_per_tour(T) * kSlotStride * sizeof(long long));
    b += align256(units * sizeof(int));
    b += align256(2 * sizeof(int));
    b += align256((size_t)kFallbackBlocks * kWave * ((size_t)max_len + 1) * sizeof(int));
    b += align256((size_t)T * sizeof(int));
    if (ordered) {
        b += align256((size_t)num_tiles(S));
        b += align256((size_t)T * (size_t)S * (size_t)ordered_pitch(max_len));
    }
    return b;
}

Workspace carve_workspace(void *base, int32_t T, int32_t max_len, int32_t N, int64_t S,
                          bool ordered)
{
    (void)N;
    const size_t units = (size_t)T * (size_t)num_tiles(S);
    char *p = static_cast<char *>(base);
    Workspace ws;
    ws.tab = reinterpret_cast<int2 *>(p);
    p += align256((size_t)T * ((size_t)max_len + kTabPad) * sizeof(int2));
    ws.ab = reinterpret_cast<int2 *>(p);
    p += align256((size_t)T * max_len * sizeof(int2));
    ws.rec = reinterpret_cast<TourRec *>(p);
    p += align256((size_t)T * sizeof(TourRec));
    ws.slots = reinterpret_cast<long long *>(p);
    p += align256((size_t)T * slots_per_tour(T) * kSlotStride * sizeof(long long));
    ws.list = reinterpret_cast<int *>(p);
    p += align256(units * sizeof(int));
    ws.list_count = reinterpret_cast<int *>(p);
    ws.done = ws.list_count + 1;
    p += align256(2 * sizeof(int));
    ws.vscratch = reinterpret_cast<int *>(p);
    p += align256((size_t)kFallbackBlocks * kWave * ((size_t)max_len + 1) * sizeof(int));
    ws.order = reinterpret_cast<int *>(p);
    p += align256((size_t)T * sizeof(int));
    ws.tile_bad = nullptr;
    ws.perm = nullptr;
    if (ordered) {
        ws.tile_bad = reinterpret_cast<uint8_t *>(p);
        p += align256((size_t)num_tiles(S));
        ws.perm = reinterpret_cast<uint8_t *>(p);
    }
    ws.max_len = max_len;
    return ws;
}

Schedule default_schedule(int32_t N, int64_t S, int32_t Q)
{
    (void)N;
    (void)S;
    Schedule s;
    s.ring = Q > 200 ? 64 : 32;
    s.first = Q > 200 ? 16 : Q > 100 ? 8 : 6;
    s.group = Q > 200 ? 4 : 3;
    s.every = Q > 200 ? 4 : 3;
    s.waves = 0;
    s.path = 0;
    return s;
}

int compiled_schedules(Schedule *out, int cap)
{
    int n = 0;
#define SPLIT_LIST(R_, F_, G_, E_)                                                               \
    if (n < cap)                                                                                 \
        out[n] = Schedule{R_, F_, G_, E_, 0, 0};                                                 \
    ++n;
    SPLIT_WINDOW_VARIANTS(SPLIT_LIST)
#undef SPLIT_LIST
    return n;
}

bool schedule_supported(const Schedule &s)
{
#define SPLIT_SUPPORTED(R_, F_, G_, E_)                                                          \
    if (s.ring == R_ && s.first == F_ && s.group == G_ && s.every == E_)                         \
        return true;
    SPLIT_WINDOW_VARIANTS(SPLIT_SUPPORTED)
#undef SPLIT_SUPPORTED
    return false;
}

hipError_t launch_permute(const int16_t *demands, int32_t N, int64_t S, int32_t T,
                          int32_t max_len, const Workspace &ws, hipStream_t stream)
{
    static bool perm_attr = false;
    if (!perm_attr) {
        const hipError_t e =
            hipFuncSetAttribute(reinterpret_cast<const void *>(&permute_tile_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLdsLimit);
        if (e != hipSuccess)
            return e;
        perm_attr = true;
    }
    hipLaunchKernelGGL(permute_tile_kernel, dim3((unsigned)num_tiles(S)), dim3(kPermThreads),
                       permute_lds_bytes(N, max_len), stream, demands, N, S, T,
                       ordered_pitch(max_len), ws);
    return hipGetLastError();
}

constexpr int64_t kOrderMaxDemandBytes = 64ll << 20;

template <int R, int F, int G, int E>
static hipError_t launch_tiles(const int16_t *demands, int32_t N, int64_t S, int32_t Q, int32_t T,
                               const int32_t *lens, int32_t *costs, const Workspace &ws,
                               hipStream_t stream, int W)
{
    const int NG = (T + W - 1) / W;
    const int64_t groups = (int64_t)NG * num_tiles(S);
    const size_t lds = (((size_t)kTile * (size_t)N + 15) & ~(size_t)15) + 16; // rows + flag
    static int lds_limit = -1;
    if (lds_limit < 0) {
        int dev = 0, lim = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess)
            return e;
        lim = lim < kLdsLimit ? lim : kLdsLimit;
        e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&split_tile_kernel<R, F, G, E, kStageBatch>),
            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(
                reinterpret_cast<const void *>(&split_tile_kernel<R, F, G, E, kTileStageBatch>),
                hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e != hipSuccess)
            return e;
        lds_limit = lim;
    }
    const int use_lds = lds <= (size_t)lds_limit ? 1 : 0;
    const size_t lds_bytes = use_lds ? lds : 0;
    // Ragged tours in decreasing length when there are several groups and
    // the demand matrix is small enough to stay in the last-level cache
    // while every group stages its copy of a tile.
    const int by_length = lens && NG > 1 && T <= kOrderMaxTours &&
                                  (int64_t)S * N * (int64_t)sizeof(int16_t) <= kOrderMaxDemandBytes
                              ? 1
                              : 0;
    if (by_length) {
        hipLaunchKernelGGL(order_kernel, dim3(1), dim3(kOrderThreads), 0, stream, lens, T,
                           ws.max_len, ws.order);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    // the larger staging batch where LDS caps a CU at 12 one-wave
    // workgroups (three per SIMD) anyway
    const bool wide_stage = W == 1 && use_lds && (size_t)kLdsLimit / lds <= 12;
    if (wide_stage)
        hipLaunchKernelGGL((split_tile_kernel<R, F, G, E, kTileStageBatch>), dim3((unsigned)groups),
                           dim3(kWave * W), lds_bytes, stream, demands, N, S, Q, T, costs, ws,
                           use_lds, by_length);
    else
        hipLaunchKernelGGL((split_tile_kernel<R, F, G, E, kStageBatch>), dim3((unsigned)groups),
                           dim3(kWave * W), lds_bytes, stream, demands, N, S, Q, T, costs, ws,
                           use_lds, by_length);
    return hipGetLastError();
}

hipError_t launch_eval(const int32_t *tours, const int32_t *lens, int32_t T, int32_t max_len,
                       const int32_t *dist, int32_t N, const int16_t *demands, int64_t S,
                       int32_t Q, int32_t *costs, int64_t *sums, double *means,
                       const Workspace &ws, hipStream_t stream, const Schedule &sched,
                       const LaunchEvents *ev)
{
    if (!schedule_supported(sched))
        return hipErrorInvalidValue;
    hipError_t e = launch_prep(tours, lens, T, max_len, dist, N, ws, stream);
    if (e != hipSuccess)
        return e;
    if (ev && ev->before) {
        e = hipEventRecord(ev->before, stream);
        if (e != hipSuccess)
            return e;
    }
    if (ws.perm) {
        e = launch_permute(demands, N, S, T, max_len, ws, stream);
        if (e != hipSuccess)
            return e;
        const int32_t pitch = ordered_pitch(max_len);
        const int64_t units = (int64_t)T * num_tiles(S);
#define SPLIT_LAUNCH_O(R_, F_, G_, E_)                                                           \
    if (sched.ring == R_ && sched.first == F_ && sched.group == G_ && sched.every == E_)          \
        hipLaunchKernelGGL((split_ordered_kernel<R_, F_, G_, E_>), dim3((unsigned)units),          \
                           dim3(kWave), 0, stream, S, Q, T, pitch, costs, ws);
        SPLIT_WINDOW_VARIANTS(SPLIT_LAUNCH_O)
#undef SPLIT_LAUNCH_O
        e = hipGetLastError();
    } else {
#define SPLIT_LAUNCH(R_, F_, G_, E_)                                                             \
    if (sched.ring == R_ && sched.first == F_ && sched.group == G_ && sched.every == E_)          \
        e = launch_tiles<R_, F_, G_, E_>(demands, N, S, Q, T, lens, costs, ws, stream,            \
                                         sched.waves ? sched.waves : waves_per_group(T, N));
        SPLIT_WINDOW_VARIANTS(SPLIT_LAUNCH)
#undef SPLIT_LAUNCH
    }
    if (e != hipSuccess)
        return e;
    if (ev && ev->after) {
        e = hipEventRecord(ev->after, stream);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(fallback_final_kernel, dim3(kFallbackBlocks), dim3(kWave), 0, stream,
                       demands, N, S, Q, T, costs, sums, means, ws);
    return hipGetLastError();
}

hipError_t launch_count_mismatch(const int32_t *a, const int32_t *b, int64_t n, int64_t *out,
                                 hipStream_t stream)
{
    hipLaunchKernelGGL(zero_i64_kernel, dim3(1), dim3(64), 0, stream, out, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int64_t blocks = n / (256 * 16) + 1 < 2048 ? n / (256 * 16) + 1 : 2048;
    hipLaunchKernelGGL(count_mismatch_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a, b,
                       n, reinterpret_cast<unsigned long long *>(out));
    return hipGetLastError();
}

hipError_t launch_count_cells(const int32_t *tours, const int32_t *lens, int32_t T, int32_t N,
                              const int16_t *demands, int64_t S, int32_t Q, int64_t *cells,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(zero_i64_kernel, dim3((T + 255) / 256), dim3(256), 0, stream, cells, T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int64_t units = (int64_t)T * num_tiles(S);
    hipLaunchKernelGGL(count_cells_kernel, dim3((unsigned)units), dim3(kWave), 0, stream, tours,
                       lens, T, N, demands, S, Q, reinterpret_cast<unsigned long long *>(cells));
    return hipGetLastError();
}

} // namespace splitk
