// split_minplus.hip -- the generic stage-wise Bellman update in the
// (min, +) semiring (Sec. 2, "Min-Plus Matrix Formulation"; App. A,
// "Illustrative example for the min-plus matrix-vector Bellman update";
// the scenario-batched forward DP of App. A), with recorded minimisers and
// backtracking (App. B: the batched DP records its minimisers and is
// backtracked to recover decisions), and the transition generator of the
// order-up-to inventory instance (App. B, its illustrative matrix form).
//
//   J_{t+1}(j) = min_i A_t(i, j) + J_t(i),   t = 0..T-1,
//
// for a batch of B independent problems (scenarios, or customer-scenario
// pairs) with m states per stage.  Values are non-negative int32; INT32_MAX
// is +inf, and a finite sum that reaches it is +inf (the sum of two values
// in [0, 2^31 - 1] fits 32 unsigned bits, so one unsigned add and one
// unsigned min against INT32_MAX give the saturated sum; a negative input
// reads as +inf).
//
// Layout: one wave per batch element, its J in LDS (double buffer); lane j
// owns target state j (and j + 64, ...) and reads J_t(i) as an LDS
// broadcast.  Up to 32 states each stage's matrix is staged in LDS with
// full-wave dword loads issued one stage ahead; larger ones are read column
// by column from global memory (row i of A_t is contiguous, so each row read is coalesced
// across lanes).  With A per element the update streams T * m * m * 4
// bytes per element: HBM-bound.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "split_device.h"
#include "split_eval.h"
#include "split_minplus.h"

namespace splitk {

namespace {

constexpr uint32_t kMpInf = 0x7FFFFFFFu;

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b)
{
    // a, b <= kMpInf (after clamping): the 32-bit sum cannot wrap
    return min(a + b, kMpInf);
}

// grid = B waves; LDS: 2 * m int32
__global__ __launch_bounds__(kWave) void minplus_forward_kernel(
    const int32_t *__restrict__ A, int32_t shared, int32_t T, int32_t m, int64_t B,
    const int32_t *__restrict__ J0, int32_t *__restrict__ JT, int32_t *__restrict__ arg)
{
    extern __shared__ uint32_t jbuf[];
    const int64_t b = blockIdx.x;
    const int lane = threadIdx.x;
    uint32_t *cur = jbuf, *nxt = jbuf + m;
    for (int j = lane; j < m; j += kWave)
        cur[j] = min((uint32_t)J0[b * m + j], kMpInf);
    __syncthreads();
    const int64_t mm = (int64_t)m * m;
    for (int t = 0; t < T; ++t) {
        const uint32_t *At = reinterpret_cast<const uint32_t *>(
            shared ? A + (int64_t)t * mm : A + ((int64_t)t * B + b) * mm);
        for (int j = lane; j < m; j += kWave) {
            uint32_t best = kMpInf;
            int bi = -1;
            int i = 0;
            for (; i + 4 <= m; i += 4) {
                uint32_t a[4], c[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    a[u] = min(At[(int64_t)(i + u) * m + j], kMpInf);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    c[u] = sat_add(a[u], cur[i + u]);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (c[u] < best) { // strict: the smallest i keeps a tie
                        best = c[u];
                        bi = i + u;
                    }
            }
            for (; i < m; ++i) {
                const uint32_t c = sat_add(min(At[(int64_t)i * m + j], kMpInf), cur[i]);
                if (c < best) {
                    best = c;
                    bi = i;
                }
            }
            nxt[j] = best;
            if (arg)
                arg[((int64_t)t * B + b) * m + j] = best < kMpInf ? bi : -1;
        }
        __syncthreads();
        uint32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    for (int j = lane; j < m; j += kWave)
        JT[b * m + j] = (int32_t)cur[j];
}

// Small state spaces (m <= 32): each stage's matrix (m*m <= 1024 int32,
// contiguous) is read with all 64 lanes loading consecutive dwords into
// registers one stage ahead, stored to LDS, and the update reads it from
// there, so the loads of stage t+1 are in flight while stage t is relaxed.
// grid = B waves; LDS: (2m + m*m) int32.
constexpr int kStagedMaxStates = 32;
constexpr int kStagedRegs = kStagedMaxStates * kStagedMaxStates / 64; // dwords per lane

__global__ __launch_bounds__(kWave) void minplus_forward_staged_kernel(
    const int32_t *__restrict__ A, int32_t shared, int32_t T, int32_t m, int64_t B,
    const int32_t *__restrict__ J0, int32_t *__restrict__ JT, int32_t *__restrict__ arg)
{
    extern __shared__ uint32_t sm[];
    const int64_t b = blockIdx.x;
    const int lane = threadIdx.x;
    uint32_t *cur = sm, *nxt = sm + m, *sA = sm + 2 * m;
    const int mm = m * m;
    auto stage_ptr = [&](int t) {
        return reinterpret_cast<const uint32_t *>(shared ? A + (int64_t)t * mm
                                                         : A + ((int64_t)t * B + b) * mm);
    };
    for (int j = lane; j < m; j += kWave)
        cur[j] = min((uint32_t)J0[b * m + j], kMpInf);
    uint32_t pre[kStagedRegs];
    {
        const uint32_t *A0 = stage_ptr(0);
#pragma unroll
        for (int c = 0; c < kStagedRegs; ++c) {
            const int e = lane + kWave * c;
            pre[c] = e < mm ? A0[e] : 0u;
        }
    }
    for (int t = 0; t < T; ++t) {
#pragma unroll
        for (int c = 0; c < kStagedRegs; ++c) {
            const int e = lane + kWave * c;
            if (e < mm)
                sA[e] = min(pre[c], kMpInf);
        }
        __syncthreads();
        if (t + 1 < T) { // next stage's matrix, in flight during this stage
            const uint32_t *An = stage_ptr(t + 1);
#pragma unroll
            for (int c = 0; c < kStagedRegs; ++c) {
                const int e = lane + kWave * c;
                pre[c] = e < mm ? An[e] : 0u;
            }
        }
        if (lane < m) {
            const int j = lane;
            uint32_t best = kMpInf;
            int bi = -1;
            for (int i = 0; i < m; ++i) {
                const uint32_t c = sat_add(sA[i * m + j], cur[i]);
                if (c < best) { // strict: the smallest i keeps a tie
                    best = c;
                    bi = i;
                }
            }
            nxt[j] = best;
            if (arg)
                arg[((int64_t)t * B + b) * m + j] = best < kMpInf ? bi : -1;
        }
        __syncthreads();
        uint32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    for (int j = lane; j < m; j += kWave)
        JT[b * m + j] = (int32_t)cur[j];
}

// one thread per element: the smallest minimising final state, then back
// through the recorded minimisers; -1 throughout when J_T is all +inf
__global__ void minplus_backtrack_kernel(const int32_t *__restrict__ JT,
                                         const int32_t *__restrict__ arg, int32_t T, int32_t m,
                                         int64_t B, int32_t *__restrict__ path)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B)
        return;
    uint32_t best = kMpInf;
    int s = -1;
    for (int j = 0; j < m; ++j) {
        const uint32_t v = (uint32_t)JT[b * m + j];
        if (v < best) {
            best = v;
            s = j;
        }
    }
    path[(int64_t)T * B + b] = s;
    for (int t = T - 1; t >= 0; --t) {
        if (s >= 0) {
            s = arg[((int64_t)t * B + b) * m + s];
            if (s < -1 || s >= m)
                s = -1; // not a recorded minimiser (cannot happen for a finite J_T)
        }
        path[(int64_t)t * B + b] = s;
    }
}

// One wave per (day, problem) pair tb = t*B + b (striding past 2^20): the
// cheapest route option with room for each delivery size q (LDS), then the
// lanes write the entries A(I, J) of its matrix in row-major order
// (coalesced).  Entry e = lane + 64k has the same (I, J) in every matrix, so
// each lane steps its (I, J) by 64 entries without a division; h sits in LDS.
// Measured alternatives: persistent waves over many pairs (each wave then
// serialises its load latencies) and per-lane option scans without LDS
// (dependent loads per entry) were both slower.
constexpr int kGenThreads = 64;

__global__ __launch_bounds__(kGenThreads) void ou_transitions_kernel(
    int32_t U, int64_t TB, int32_t R, const int32_t *__restrict__ demand,
    const int32_t *__restrict__ opt_cost, const int32_t *__restrict__ opt_cap,
    const int32_t *__restrict__ h, int32_t u, int32_t rho, int32_t *__restrict__ A)
{
    extern __shared__ long long tr[]; // transport(q), q = 0..U (kMpInf: impossible); then h
    const int m = U + 1;
    int32_t *hs = reinterpret_cast<int32_t *>(tr + m);
    for (int J = threadIdx.x; J < m; J += blockDim.x)
        hs[J] = h[J];
    const int mm = m * m;
    const int I0 = (int)threadIdx.x / m, J0 = (int)threadIdx.x - I0 * m;
    const int dI = kGenThreads / m, dJ = kGenThreads - dI * m;
    for (int64_t tb = blockIdx.x; tb < TB; tb += gridDim.x) {
        __syncthreads();
        for (int q = threadIdx.x; q < m; q += blockDim.x) {
            long long c = q == 0 ? 0 : (long long)kMpInf;
            for (int r = 0; q > 0 && r < R; ++r)
                if (opt_cap[tb * R + r] >= q)
                    c = min(c, (long long)opt_cost[tb * R + r]);
            tr[q] = c >= kMpInf ? (long long)kMpInf : c + (long long)u * q;
        }
        __syncthreads();
        const int d = demand[tb];
        const long long deliver_left = (long long)rho * max(0, d - U); // shortage after delivering
        const int Jd = max(0, U - d);                                   // level after delivering
        int32_t *out = A + tb * (int64_t)mm;
        int I = I0, J = J0;
        for (int e = threadIdx.x; e < mm; e += kGenThreads) {
            long long best = kMpInf;
            // no delivery
            if (max(0, I - d) == J)
                best = (long long)hs[J] + (long long)rho * max(0, d - I);
            // deliver up to U (a distinct choice only when I < U)
            const int q = U - I;
            if (q > 0 && J == Jd && tr[q] < kMpInf)
                best = min(best, tr[q] + hs[J] + deliver_left);
            out[e] = (int32_t)min(best, (long long)kMpInf);
            I += dI;
            J += dJ;
            if (J >= m) {
                J -= m;
                ++I;
            }
        }
    }
}

} // namespace

hipError_t launch_minplus_forward(const int32_t *A, int32_t shared, int32_t T, int32_t m,
                                  int64_t B, const int32_t *J0, int32_t *JT, int32_t *arg,
                                  hipStream_t stream)
{
    if (m <= kStagedMaxStates)
        hipLaunchKernelGGL(minplus_forward_staged_kernel, dim3((unsigned)B), dim3(kWave),
                           (size_t)(2 * m + m * m) * sizeof(uint32_t), stream, A, shared, T, m, B,
                           J0, JT, arg);
    else
        hipLaunchKernelGGL(minplus_forward_kernel, dim3((unsigned)B), dim3(kWave),
                           (size_t)2 * m * sizeof(uint32_t), stream, A, shared, T, m, B, J0, JT,
                           arg);
    return hipGetLastError();
}

hipError_t launch_minplus_backtrack(const int32_t *JT, const int32_t *arg, int32_t T, int32_t m,
                                    int64_t B, int32_t *path, hipStream_t stream)
{
    const unsigned blocks = (unsigned)((B + 255) / 256);
    hipLaunchKernelGGL(minplus_backtrack_kernel, dim3(blocks), dim3(256), 0, stream, JT, arg, T, m,
                       B, path);
    return hipGetLastError();
}

hipError_t launch_ou_transitions(int32_t U, int32_t T, int64_t B, int32_t R,
                                 const int32_t *demand, const int32_t *opt_cost,
                                 const int32_t *opt_cap, const int32_t *h, int32_t u, int32_t rho,
                                 int32_t *A, hipStream_t stream)
{
    const int64_t TB = (int64_t)T * B;
    // one wave per pair (a persistent grid serialises each wave's global
    // load latencies over its pairs: measured slower)
    const int64_t blocks = TB < (1 << 20) ? TB : (1 << 20);
    hipLaunchKernelGGL(ou_transitions_kernel, dim3((unsigned)blocks), dim3(kGenThreads),
                       ((size_t)U + 1) * (sizeof(long long) + sizeof(int32_t)), stream, U, TB, R,
                       demand, opt_cost, opt_cap, h, u, rho, A);
    return hipGetLastError();
}

} // namespace splitk
