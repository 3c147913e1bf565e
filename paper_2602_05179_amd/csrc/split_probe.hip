// split_probe.hip -- measured int32 VALU rate of the device (a roofline
// reference for the evaluation kernels; not part of the method).
//
// Every lane runs eight independent dependency chains of v_min_i32, so the
// wave never waits on its own results; the grid puts eight waves on every
// SIMD.  The rate is lane-operations per second over the timed launch.

#include <hip/hip_runtime.h>

#include "split_eval.h"
#include "split_internal.h"

namespace splitk {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeIters = 4096;
constexpr int kProbeOpsPerIter = 64; // 8 chains x 8 steps

__global__ __launch_bounds__(kProbeThreads) void valu_probe_kernel(int *out, int iters)
{
    int a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3;
    int a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    const int b = blockIdx.x;
    for (int it = 0; it < iters; ++it) {
#define SPLIT_PROBE_STEP                                                                          \
    "v_min_i32_e32 %0, %0, %8\n\tv_min_i32_e32 %1, %1, %8\n\tv_min_i32_e32 %2, %2, %8\n\t"        \
    "v_min_i32_e32 %3, %3, %8\n\tv_min_i32_e32 %4, %4, %8\n\tv_min_i32_e32 %5, %5, %8\n\t"        \
    "v_min_i32_e32 %6, %6, %8\n\tv_min_i32_e32 %7, %7, %8\n\t"
        asm volatile(SPLIT_PROBE_STEP SPLIT_PROBE_STEP SPLIT_PROBE_STEP SPLIT_PROBE_STEP
                         SPLIT_PROBE_STEP SPLIT_PROBE_STEP SPLIT_PROBE_STEP SPLIT_PROBE_STEP
                     : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6),
                       "+v"(a7)
                     : "v"(b));
#undef SPLIT_PROBE_STEP
    }
    const int r = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
    if (r == 0x7fffffff)
        out[0] = r; // keeps the chains live; never true for these inputs
}

} // namespace

} // namespace splitk

extern "C" int split_probe_valu_peak(double *lane_ops_per_s, split_stream_t stream)
{
    using namespace splitk;
    clear_error();
    if (!lane_ops_per_s)
        return set_error(SPLIT_EINVAL, "null pointer argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return set_error(SPLIT_EDEVICE, "device query: %s", hipGetErrorString(e));
    // eight waves per SIMD: 4 SIMDs x 8 waves x 64 lanes per CU
    const int blocks = cus * 4 * 8 * 64 / kProbeThreads;
    int *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f;
    int rc = SPLIT_OK;
    if (hipMalloc(&out, sizeof(int)) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = set_error(SPLIT_ENOMEM, "probe buffers");
        goto done;
    }
    hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0, st, out,
                       kProbeIters / 8); // warm-up
    e = hipEventRecord(e0, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0, st, out,
                           kProbeIters);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipEventRecord(e1, st);
    if (e == hipSuccess)
        e = hipEventSynchronize(e1);
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess || ms <= 0.f) {
        rc = set_error(SPLIT_EDEVICE, "probe launch: %s", hipGetErrorString(e));
        goto done;
    }
    *lane_ops_per_s = (double)blocks * kProbeThreads * (double)kProbeIters * kProbeOpsPerIter /
                      (ms * 1e-3);
done:
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (out)
        (void)hipFree(out);
    return rc;
}
