// split_small.hip -- the whole evaluation of one short tour over a few
// thousand scenarios in ONE launch of one workgroup: the latency form of
// the plain split (the recursion of Sec. 2.3 per scenario, then the SAA
// mean over the scenarios).
//
// For small problems the three launches of the general path (per-tour
// tables, tiles, exact fallback with the final fold) cost more than the
// work itself.  Here the waves of one workgroup first build the tour's
// tables together (the general tables' arithmetic and validation for one
// tour, one position per thread), then each wave takes 64-scenario tiles
// in turn (tile staged in its own LDS region, the register-ring recursion,
// the exact recursion inline for a tile whose windows leave the ring or
// whose demands do not fit a byte), and the workgroup folds the exact sum
// and writes the mean.  Costs, sums and means are identical to the general
// path's for the same inputs.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "split_device.h"
#include "split_dp.h"
#include "split_eval.h"
#include "split_internal.h"
#include "split_small.h"

namespace splitk {

namespace {

// workgroup size: eight waves (two per SIMD) leave each lane the registers
// of the recursion without spills (sixteen waves cap them at 128, below
// what either ring length needs)
template <int R> __host__ __device__ constexpr int small_threads() { return 512; }

__host__ __device__ inline size_t small_row_bytes(int32_t N) { return (((size_t)kTile * (size_t)N + 15) & ~(size_t)15) + 16; }

// The tour's tables and record as the general per-tour pass computes them
// for one tour: tab = {customer index, c_j} for positions 1..n with zero
// padding, ab = {a_j, b_j}, and the validation (customer ids, costs in
// range, the exactness guard 3 n max_cost < 2^29).  One position per
// thread (n <= THREADS).
template <int THREADS>
__device__ __forceinline__ TourRec small_prep(const int32_t *__restrict__ tours, int32_t n_in,
                                              int32_t max_len, const int32_t *__restrict__ dist,
                                              int32_t N, const Workspace &ws)
{
    constexpr int kWaves = THREADS / kWave;
    __shared__ long long s_scan[kWaves];
    __shared__ int s_bad[kWaves], s_max[kWaves];
    __shared__ int s_first;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int64_t N1 = (int64_t)N + 1;
    int bad = (n_in < 0 || n_in > max_len) ? 1 : 0;
    const int nn = bad ? 0 : n_in;
    int2 *tab = ws.tab;
    int2 *ab = ws.ab;
    if (tid < kTabPad)
        tab[tid == 0 ? 0 : nn + tid] = make_int2(0, 0);
    if (tid == 0)
        s_first = 0;
    __syncthreads();
    const int k = tid; // tour position k+1
    long long arc = 0;
    int c = 0, out = 0, in = 0, cn = 0, outn = 0, a = 0, maxc = 0;
    if (k < nn) {
        c = tours[k];
        if (c < 1 || c > N) {
            bad = 1;
            c = 1;
        }
        out = dist[c];
        in = dist[(int64_t)c * N1];
        if (k + 1 < nn) {
            cn = tours[k + 1];
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
        maxc = max(out, max(in, a));
        if (k == 0)
            s_first = out; // a_1 = c[0][sigma_1] since D_1 = 0
    }
    // exclusive prefix of the arcs: D_{k+1} = sum over m < k of arc_m
    long long incl = arc;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const long long y = __shfl_up(incl, o, kWave);
        if (lane >= o)
            incl += y;
    }
    int b = bad, mc = maxc;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        b |= __shfl_xor(b, o, kWave);
        mc = max(mc, __shfl_xor(mc, o, kWave));
    }
    if (lane == kWave - 1)
        s_scan[wid] = incl;
    if (lane == 0) {
        s_bad[wid] = b;
        s_max[wid] = mc;
    }
    __syncthreads();
    long long pre = 0;
    for (int w = 0; w < wid; ++w)
        pre += s_scan[w];
    const long long Dk = pre + incl - arc;
    if (k < nn) {
        const int ck = (k + 1 < nn) ? (in + outn - (int)arc) : 0;
        tab[k + 1] = make_int2(c - 1, ck);
        ab[k] = make_int2((int)((long long)out - Dk), (int)(Dk + in));
    }
    int allbad = 0, allmax = 0;
    for (int w = 0; w < kWaves; ++w) {
        allbad |= s_bad[w];
        allmax = max(allmax, s_max[w]);
    }
    if ((long long)3 * nn * allmax >= (1LL << 29))
        allbad = 1;
    // the tables are complete in memory before any wave reads them
    __threadfence();
    __syncthreads();
    TourRec rec;
    rec.n = nn;
    rec.f0 = s_first;
    rec.bn = nn > 0 ? ab[nn - 1].y : 0; // b_n
    rec.status = allbad ? ST_BAD_TOUR : ST_OK;
    rec.maxc = allmax;
    return rec;
}

template <int R, int F, int G, int E>
__global__ __launch_bounds__(small_threads<R>()) void small_kernel(
    const int32_t *__restrict__ tours, const int32_t *__restrict__ lens, int32_t max_len,
    const int32_t *__restrict__ dist, int32_t N, const int16_t *__restrict__ demands, int64_t S,
    int32_t Q, int32_t *__restrict__ costs, int64_t *__restrict__ sums,
    double *__restrict__ means, Workspace ws)
{
    constexpr int THREADS = small_threads<R>();
    constexpr int kWaves = THREADS / kWave;
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ long long s_sum[kWaves];
    __shared__ int s_ninf[kWaves], s_neg[kWaves];
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const TourRec rec = small_prep<THREADS>(tours, lens ? lens[0] : max_len, max_len, dist, N, ws);
    const int n = __builtin_amdgcn_readfirstlane(rec.n);
    const bool valid = rec.status == ST_OK;
    // The recursion reads the table through scalar loads, which the
    // compiler may move freely (it takes such memory as unchanging during
    // the kernel); the empty asm hands over the pointer only after the
    // barrier that completes the table, so no read of it can move above.
    const int2 *tabg = ws.tab;
    asm volatile("" : "+s"(tabg));
    CInt *tab = (CInt *)tabg;
    const int64_t tiles = (S + kWave - 1) / kWave;
    const size_t region = small_row_bytes(N);
    uint8_t *my = lds + (size_t)w * region;
    int &s_bad = *reinterpret_cast<int *>(my + region - 16);
    int *V = ws.vscratch + (int64_t)w * kWave * (ws.max_len + 1);
    long long sum = 0;
    int ninf = 0;
    bool neg = false;
    const int trips = (int)((tiles + kWaves - 1) / kWaves); // the same for every wave
    for (int it = 0; it < trips; ++it) {
        const int64_t k = (int64_t)it * kWaves + w;
        const int64_t s0 = k * kWave;
        const int rows = k < tiles ? (int)min<int64_t>(kWave, S - s0) : 0;
        // every wave stages (possibly nothing) so the barriers inside match
        const bool ok = stage_tile_u8(demands + (rows ? s0 * N : 0), my, (int64_t)rows * N, lane,
                                      kWave, s_bad);
        if (rows == 0)
            continue;
        int v = 0;
        if (valid && n > 0) {
            bool ovf = false;
            if (ok && lane < rows)
                v = dp_lane<R, F, G, E>(my + (int64_t)lane * N, tab, n, rec.f0, Q, ovf) +
                    rec.bn;
            if (!ok || ballot(ovf) != 0) {
                bool negq = false;
                v = 0;
                if (lane < rows)
                    v = exact_lane(demands + (s0 + lane) * N, ws.tab, ws.ab, n, Q, V, lane, negq);
                neg = neg || ballot(negq) != 0;
            }
        }
        const bool inf = lane < rows && (!valid || v >= kInf);
        const bool fin = lane < rows && !inf;
        if (lane < rows)
            costs[s0 + lane] = inf ? SPLIT_INF : v;
        sum += wave_sum_i64(fin ? (long long)v : 0LL);
        ninf += wave_sum_i32(inf ? 1 : 0);
    }
    if (lane == 0) {
        s_sum[w] = sum;
        s_ninf[w] = ninf;
        s_neg[w] = neg ? 1 : 0;
    }
    __syncthreads();
    long long tot = 0, ni = 0;
    int anyneg = 0;
    for (int q = 0; q < kWaves; ++q) {
        tot += s_sum[q];
        ni += s_ninf[q];
        anyneg |= s_neg[q];
    }
    // an invalid tour, or a negative demand met by the recursion: the sum
    // is invalid and every cost SPLIT_INF
    const bool bad = !valid || anyneg;
    if (tid == 0) {
        if (bad) {
            sums[0] = SPLIT_SUM_INVALID;
            means[0] = __builtin_nan("");
        } else if (ni) {
            sums[0] = INT64_MAX;
            means[0] = __builtin_inf();
        } else {
            sums[0] = tot;
            means[0] = (double)tot / (double)S;
        }
    }
    if (bad)
        for (int64_t i = tid; i < S; i += THREADS)
            costs[i] = SPLIT_INF;
}

static_assert((size_t)(small_threads<32>() / kWave) * (((size_t)kTile * kSmallMaxN + 15) / 16 * 16 + 16) +
                      1024 <=
                  (size_t)kLdsLimit,
              "staged tiles and the static LDS of the one-launch form exceed a workgroup's LDS");

template <int R, int F, int G, int E>
hipError_t launch_small_t(const int32_t *tours, const int32_t *lens, int32_t max_len,
                          const int32_t *dist, int32_t N, const int16_t *demands, int64_t S,
                          int32_t Q, int32_t *costs, int64_t *sums, double *means,
                          const Workspace &ws, hipStream_t stream)
{
    constexpr int THREADS = small_threads<R>();
    const size_t lds = (size_t)(THREADS / kWave) * small_row_bytes(N);
    hipLaunchKernelGGL((small_kernel<R, F, G, E>), dim3(1), dim3(THREADS), lds, stream, tours,
                       lens, max_len, dist, N, demands, S, Q, costs, sums, means, ws);
    return hipGetLastError();
}

} // namespace

hipError_t small_prepare()
{
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        const int bytes = (int)((size_t)(small_threads<32>() / kWave) * small_row_bytes(kSmallMaxN));
#define SPLIT_SMALL_ATTR(R_, F_, G_, E_)                                                         \
    if (err == hipSuccess)                                                                       \
        err = hipFuncSetAttribute(reinterpret_cast<const void *>(&small_kernel<R_, F_, G_, E_>),   \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        SPLIT_WINDOW_VARIANTS(SPLIT_SMALL_ATTR)
#undef SPLIT_SMALL_ATTR
    });
    return err;
}

bool small_path_fits(int32_t num_tours, int32_t max_len, int32_t N, int64_t S,
                     const Schedule &s, bool ordered)
{
    if (num_tours != 1 || ordered || s.path != 0 || !schedule_supported(s))
        return false;
    const int threads = s.ring == 64 ? small_threads<64>() : small_threads<32>();
    const int waves = threads / kWave;
    const int64_t tiles = (S + kWave - 1) / kWave;
    const int64_t per_wave = (tiles + waves - 1) / waves;
    return max_len >= 1 && max_len <= threads && N >= 1 && N <= kSmallMaxN && S >= 1 &&
           per_wave * max_len <= kSmallMaxSteps;
}

hipError_t launch_small(const int32_t *tours, const int32_t *lens, int32_t max_len,
                        const int32_t *dist, int32_t N, const int16_t *demands, int64_t S,
                        int32_t Q, int32_t *costs, int64_t *sums, double *means,
                        const Workspace &ws, hipStream_t stream, const Schedule &s)
{
    const hipError_t e = small_prepare();
    if (e != hipSuccess)
        return e;
#define SPLIT_SMALL(R_, F_, G_, E_)                                                              \
    if (s.ring == R_ && s.first == F_ && s.group == G_ && s.every == E_)                         \
        return launch_small_t<R_, F_, G_, E_>(tours, lens, max_len, dist, N, demands, S, Q, costs, \
                                              sums, means, ws, stream);
    SPLIT_WINDOW_VARIANTS(SPLIT_SMALL)
#undef SPLIT_SMALL
    return hipErrorInvalidValue;
}

} // namespace splitk
