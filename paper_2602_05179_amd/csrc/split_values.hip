// split_values.hip -- the full value table of one giant tour over every
// scenario: V_s(j) for j = 1..n (paper Sec. 2.3 recursion; the batched DP
// of App. A returns the value array over positions and scenarios, not only
// V_s(n)).
//
// One wave per tile of 64 scenarios, one scenario per lane, the recursion
// taken exactly from its definition: for each position j the lane walks its
// predecessors p = j-1, j-2, ... while the route load stays within Q,
// reading V_s(p) back from its own column of the output.  The output is
// position-major (V[(j-1)*S + s]), so a wave's reads and writes of one
// position are one coalesced row that the recent positions keep in L2.
// Demands are read through the tour from the lane's row in global memory,
// as int16 (any value the interface accepts).  This is an opt-in output
// for inspection of the whole table; the evaluation kernels compute only
// V_s(n).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "split_device.h"
#include "split_eval.h"
#include "split_internal.h"
#include "split_values.h"

namespace splitk {

namespace {

__global__ void values_status_kernel(int32_t *status) { *status = 0; }

__global__ __launch_bounds__(kWave) void values_kernel(const int16_t *__restrict__ demands,
                                                       int32_t N, int64_t S, int32_t Q,
                                                       Workspace ws, int32_t *__restrict__ V,
                                                       int32_t *__restrict__ status)
{
    const int64_t s = (int64_t)blockIdx.x * kWave + threadIdx.x;
    const TourRec rec = ws.rec[0];
    const int n = rec.n;
    if (s >= S)
        return;
    if (rec.status != ST_OK) {
        for (int j = 1; j <= n; ++j)
            V[(int64_t)(j - 1) * S + s] = SPLIT_INF;
        return;
    }
    const int2 *__restrict__ tab = ws.tab; // {customer index, c_j}, entry j = position j
    const int2 *__restrict__ ab = ws.ab;   // {a_k, b_k}, entry k-1 = position k
    const int16_t *__restrict__ row = demands + s * N;
    bool neg = false;
    for (int j = 1; j <= n; ++j) {
        const int bj = ab[j - 1].y;
        int best = SPLIT_INF;
        int load = 0;
        for (int p = j - 1; p >= 0; --p) {
            const int q = row[tab[p + 1].x];
            neg = neg || q < 0;
            load += q;
            if (load > Q) // demands are non-negative: every longer route is too heavy
                break;
            const int vp = p == 0 ? 0 : V[(int64_t)(p - 1) * S + s];
            if (vp != SPLIT_INF)
                best = min(best, vp + ab[p].x + bj); // V(p) + W(p, j)
        }
        V[(int64_t)(j - 1) * S + s] = best;
    }
    if (neg) {
        for (int j = 1; j <= n; ++j)
            V[(int64_t)(j - 1) * S + s] = SPLIT_INF;
        atomicOr(status, 1);
    }
}

} // namespace

hipError_t launch_values(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                         const int16_t *demands, int64_t S, int32_t Q, int32_t *V,
                         int32_t *status, const Workspace &ws, hipStream_t stream)
{
    hipLaunchKernelGGL(values_status_kernel, dim3(1), dim3(1), 0, stream, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    e = launch_prep(tour, nullptr, 1, n, dist, N, ws, stream);
    if (e != hipSuccess || n == 0)
        return e;
    hipLaunchKernelGGL(values_kernel, dim3((unsigned)num_tiles(S)), dim3(kWave), 0, stream,
                       demands, N, S, Q, ws, V, status);
    return hipGetLastError();
}

} // namespace splitk
