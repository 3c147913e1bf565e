// split_ou.hip -- the order-up-to inventory DP in one kernel (App. B: each
// day a customer is replenished up to its capacity U or not at all; the
// illustrative matrix form of the DP, whose note extends the update to
// scenarios x transitions x route options with the minimum taken first over
// route options and then over predecessor states; the batched DP records
// its minimisers).
//
// For B independent problems (customer-scenario pairs) over T days with
// inventory states 0..U, the kernel computes exactly what the transition
// generator followed by the generic forward update computes,
//
//   J_{t+1}(J) = min_I  A_t(I, J) + J_t(I),
//
// without writing A_t: from inventory I with day demand d the two actions
// are "no delivery" (next level max(0, I - d), cost h[next] +
// rho * max(0, d - I)) and "deliver q = U - I" (next level max(0, U - d),
// cost transport(q) + h[next] + rho * max(0, d - U), transport(q) the
// cheapest route option whose residual capacity is at least q, plus u * q).
// So a level K >= 1 is reached without delivery from I = K + d only, level
// 0 from every I <= d, and the delivery level from every I < U.
//
// Layout: one lane per problem, its J_t in registers.  Per day a lane
//   1. takes the minimum over route options for every delivery size
//      (first reduction, over r),
//   2. folds the delivery terms of every source into one minimum with its
//      smallest minimiser, and the no-delivery terms of sources I <= d into
//      the minimum for level 0,
//   3. writes J_t(I) to its own LDS column and reads back J_t(K + d) for
//      every level K >= 1 (the shift by the lane's demand; column slots past
//      the last state hold +inf), adds h[K], and merges the delivery
//      minimum into its level (second reduction, over I; ties go to the
//      smallest I).
// Demands and option tables are read once (coalesced: a lane's R options
// are contiguous), the next day's inputs are in flight while a day is
// relaxed, and the only writes are the minimisers (optional) and J_T.
//
// Values are int32 with INT32_MAX as +inf; sums saturate at +inf (all terms
// are non-negative for valid inputs, so saturating each partial sum is
// exact).  A negative demand, option cost or h entry is invalid input: the
// kernel reports it in the status word (every access stays in bounds).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "split_device.h"
#include "split_eval.h"
#include "split_minplus.h"

namespace splitk {

namespace {

constexpr uint32_t kOuInf = 0x7FFFFFFFu;
constexpr int kOuPre = 8; // route options of the next day kept in flight

__device__ __forceinline__ uint32_t ou_sat(uint32_t a, uint32_t b)
{
    // a, b <= kOuInf: the 32-bit sum cannot wrap
    return min(a + b, kOuInf);
}

__device__ __forceinline__ uint32_t ou_clamp(uint64_t x)
{
    return x >= kOuInf ? kOuInf : (uint32_t)x;
}

__global__ __launch_bounds__(kWave) void ou_status_zero_kernel(int32_t *status)
{
    if (threadIdx.x == 0)
        *status = 0;
}

// M: compile-time bound on the states (m = U + 1 <= M).  Grid: one wave per
// 64 problems.  LDS: the lane columns (2M slots), one buffer that holds the
// option scatter and serves as the transpose buffer for coalesced reads of
// J_0 and writes of J_T and the minimisers (the 64 problems of a wave own a
// contiguous [64][m] block of each), h and the unit transport cost of every
// delivery size.
template <int M>
__global__ __launch_bounds__(kWave) void ou_dp_kernel(
    int32_t U, int32_t T, int64_t B, int32_t R, const int32_t *__restrict__ demand,
    const int32_t *__restrict__ opt_cost, const int32_t *__restrict__ opt_cap,
    const int32_t *__restrict__ h, int32_t u, int32_t rho, const int32_t *__restrict__ J0,
    int32_t *__restrict__ JT, int32_t *__restrict__ arg, int32_t *__restrict__ status)
{
    __shared__ uint32_t col[2 * M][kWave]; // col[s][lane]: J_t(s) for s < m, +inf after
    // one buffer, two uses (one wave per workgroup, so its LDS operations
    // keep program order): tm[s][lane], the cheapest route option by the
    // first source it serves (live during step 1 of a day), and xp, the
    // [lane][m] transpose buffer of J_0, J_T and the minimisers (step 3)
    __shared__ uint32_t buf[M * kWave];
    uint32_t(&tm)[M][kWave] = *reinterpret_cast<uint32_t(*)[M][kWave]>(buf);
    uint32_t *xp = buf;
    __shared__ uint32_t hs[M];
    __shared__ uint32_t uqs[M]; // u * (U - I), saturated
    const int lane = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kWave;
    const int64_t b = b0 + lane;
    const bool live = b < B;
    const int m = U + 1;
    const int rows = (int)min<int64_t>(kWave, B - b0); // problems of this wave
    const int words = rows * m;                           // contiguous words per block
    bool bad = false;
    if (lane < M) {
        const int32_t hv = lane < m ? h[lane] : 0;
        bad = hv < 0;
        hs[lane] = hv < 0 ? 0u : (uint32_t)hv; // levels past U: never added to a finite value
        uqs[lane] = lane < U ? ou_clamp((uint64_t)(uint32_t)u * (uint64_t)(U - lane)) : kOuInf;
    }
    for (int s = m; s < 2 * M; ++s)
        col[s][lane] = kOuInf;
    // J_0 of the wave's problems: coalesced words, then each lane its row
    for (int w = lane; w < words; w += kWave)
        xp[w] = min((uint32_t)J0[b0 * m + w], kOuInf);
    __syncthreads();
    uint32_t J[M];
#pragma unroll
    for (int I = 0; I < M; ++I)
        J[I] = (live && I < m) ? xp[lane * m + I] : kOuInf;

    // day 0 inputs
    int nd = 0;
    int nc[kOuPre], ncap[kOuPre];
    const int RP = R < kOuPre ? R : kOuPre;
#pragma unroll
    for (int r = 0; r < kOuPre; ++r) {
        nc[r] = 0;
        ncap[r] = -1;
    }
    if (live) {
        nd = demand[b];
#pragma unroll
        for (int r = 0; r < kOuPre; ++r)
            if (r < RP) {
                nc[r] = opt_cost[b * R + r];
                ncap[r] = opt_cap[b * R + r];
            }
    }
    for (int t = 0; t < T; ++t) {
        const int64_t tb = (int64_t)t * B + b;
        int d = nd;
        int c[kOuPre], cap[kOuPre];
#pragma unroll
        for (int r = 0; r < kOuPre; ++r) {
            c[r] = nc[r];
            cap[r] = ncap[r];
        }
        if (live && t + 1 < T) { // the next day's inputs, in flight during this day
            const int64_t tn = tb + B;
            nd = demand[tn];
#pragma unroll
            for (int r = 0; r < kOuPre; ++r)
                if (r < RP) {
                    nc[r] = opt_cost[tn * R + r];
                    ncap[r] = opt_cap[tn * R + r];
                }
        }
        bad = bad || d < 0;
        d = live ? max(d, 0) : 0;

        // 1. cheapest option with room for the delivery q = U - I of every
        //    source I < U (minimum over route options): option r serves
        //    source I when cap_r >= U - I
        //    option r serves the sources I >= U - cap_r: scatter its cost
        //    to that first source (per-lane LDS column, atomic minimum),
        //    then a prefix minimum over I
#pragma unroll
        for (int I = 0; I < M; ++I)
            tm[I][lane] = kOuInf;
#pragma unroll
        for (int r = 0; r < kOuPre; ++r) {
            if (r < RP) {
                bad = bad || (live && c[r] < 0);
                const uint32_t cr = (c[r] < 0 || !live) ? kOuInf : (uint32_t)c[r];
                const int first = max(U - cap[r], 0); // > M - 1: serves none
                if (first < M)
                    atomicMin(&tm[first][lane], cr);
            }
        }
        for (int r = kOuPre; r < R; ++r) { // options past the prefetched ones
            const int cv = live ? opt_cost[tb * R + r] : 0;
            const int kv = live ? opt_cap[tb * R + r] : -1;
            bad = bad || cv < 0;
            const uint32_t cr = cv < 0 ? kOuInf : (uint32_t)cv;
            const int first = max(U - kv, 0);
            if (first < M)
                atomicMin(&tm[first][lane], cr);
        }
        uint32_t tr[M]; // (sources I >= U have no delivery: their u * (U - I) is +inf)
        {
            uint32_t run = kOuInf;
#pragma unroll
            for (int I = 0; I < M; ++I) {
                run = min(run, tm[I][lane]);
                tr[I] = run;
            }
        }

        // 2. delivery: every source I < U lands on level Jd; no delivery:
        //    sources I <= d land on level 0 (cost h[0] + rho (d - I))
        const int Jd = max(0, U - d);
        const uint32_t dconst =
            ou_sat(hs[Jd], ou_clamp((uint64_t)(uint32_t)rho * (uint64_t)(uint32_t)max(0, d - U)));
        const uint32_t h0 = hs[0];
        uint32_t bestD = kOuInf, best0 = kOuInf;
        int argD = -1, arg0 = -1;
        // no delivery into level 0 costs h[0] + rho (d - I): in 32 bits
        // (c0 - rho I) when rho d and h[0] stay below 2^30 on every lane of
        // the wave, else exactly through the high product
        const uint32_t rd_hi = __umulhi((uint32_t)rho, (uint32_t)d);
        const uint32_t rd_lo = (uint32_t)rho * (uint32_t)d;
        const bool small = rd_hi == 0u && rd_lo < (1u << 30) && h0 < (1u << 30);
        const uint32_t c0 = h0 + rd_lo;
        // levels I >= m hold +inf throughout, so every term they give is +inf
        if (__all(small)) {
#pragma unroll
            for (int I = 0; I < M; ++I) {
                col[I][lane] = J[I];
                const uint32_t v = ou_sat(J[I], ou_sat(ou_sat(tr[I], uqs[I]), dconst));
                const bool lt = v < bestD;
                bestD = lt ? v : bestD;
                argD = lt ? I : argD;
                const uint32_t v0 = I <= d ? min(J[I] + (c0 - (uint32_t)rho * (uint32_t)I), kOuInf)
                                           : kOuInf;
                const bool lt0 = v0 < best0;
                best0 = lt0 ? v0 : best0;
                arg0 = lt0 ? I : arg0;
            }
        } else {
#pragma unroll
            for (int I = 0; I < M; ++I) {
                col[I][lane] = J[I];
                const uint32_t v = ou_sat(J[I], ou_sat(ou_sat(tr[I], uqs[I]), dconst));
                const bool lt = v < bestD;
                bestD = lt ? v : bestD;
                argD = lt ? I : argD;
                const uint32_t k = (uint32_t)max(d - I, 0);
                const uint32_t lo = (uint32_t)rho * k;
                const uint32_t hi = __umulhi((uint32_t)rho, k);
                const uint32_t sh = (hi != 0u || lo > kOuInf) ? kOuInf : lo;
                const uint32_t v0 = I <= d ? ou_sat(J[I], ou_sat(h0, sh)) : kOuInf;
                const bool lt0 = v0 < best0;
                best0 = lt0 ? v0 : best0;
                arg0 = lt0 ? I : arg0;
            }
        }

        // 3. the delivery level merged once (ties: the smallest source):
        //    its no-delivery term is J_t(Jd + d) + h[Jd] (level 0: best0)
        const int dd = d < m ? d : m; // reads past m - 1 hit the +inf slots
        uint32_t vJ = Jd == 0 ? best0 : ou_sat(col[Jd + dd][lane], hs[Jd]);
        int aJ = Jd == 0 ? arg0 : Jd + d;
        if (bestD < vJ || (bestD == vJ && argD < aJ)) {
            vJ = bestD;
            aJ = argD;
        }
        // every level: the shifted no-delivery term, or the merged value
        // (levels K >= m read +inf slots and stay +inf)
#pragma unroll
        for (int K = 0; K < M; ++K) {
            uint32_t v = K == 0 ? best0 : ou_sat(col[K + dd][lane], hs[K]);
            int a = K == 0 ? arg0 : K + d;
            const bool atJ = K == Jd;
            v = atJ ? vJ : v;
            a = atJ ? aJ : a;
            J[K] = v;
            if (K < m)
                xp[lane * m + K] = (uint32_t)(v >= kOuInf ? -1 : a);
        }
        if (arg) { // the wave's [64][m] block of day t, coalesced
            __syncthreads();
            int32_t *dst = arg + ((int64_t)t * B + b0) * m;
            for (int w = lane; w < words; w += kWave)
                dst[w] = (int32_t)xp[w];
            __syncthreads();
        }
    }
    __syncthreads();
#pragma unroll
    for (int K = 0; K < M; ++K)
        if (K < m)
            xp[lane * m + K] = J[K];
    __syncthreads();
    for (int w = lane; w < words; w += kWave)
        JT[b0 * m + w] = (int32_t)xp[w];
    if (status) {
        const uint64_t any = __ballot(bad);
        if (any != 0 && lane == __builtin_ctzll(any))
            atomicOr(status, 1);
    }
}

} // namespace

hipError_t launch_ou_dp(int32_t U, int32_t T, int64_t B, int32_t R, const int32_t *demand,
                        const int32_t *opt_cost, const int32_t *opt_cap, const int32_t *h,
                        int32_t u, int32_t rho, const int32_t *J0, int32_t *JT, int32_t *arg,
                        int32_t *status, hipStream_t stream)
{
    if (status) {
        hipLaunchKernelGGL(ou_status_zero_kernel, dim3(1), dim3(kWave), 0, stream, status);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    const unsigned blocks = (unsigned)((B + kWave - 1) / kWave);
    const int m = U + 1;
    if (m <= 8)
        hipLaunchKernelGGL(ou_dp_kernel<8>, dim3(blocks), dim3(kWave), 0, stream, U, T, B, R,
                           demand, opt_cost, opt_cap, h, u, rho, J0, JT, arg, status);
    else if (m <= 16)
        hipLaunchKernelGGL(ou_dp_kernel<16>, dim3(blocks), dim3(kWave), 0, stream, U, T, B, R,
                           demand, opt_cost, opt_cap, h, u, rho, J0, JT, arg, status);
    else if (m <= 24)
        hipLaunchKernelGGL(ou_dp_kernel<24>, dim3(blocks), dim3(kWave), 0, stream, U, T, B, R,
                           demand, opt_cost, opt_cap, h, u, rho, J0, JT, arg, status);
    else
        hipLaunchKernelGGL(ou_dp_kernel<kOuMaxStates>, dim3(blocks), dim3(kWave), 0, stream, U,
                           T, B, R, demand, opt_cost, opt_cap, h, u, rho, J0, JT, arg, status);
    return hipGetLastError();
}

} // namespace splitk
