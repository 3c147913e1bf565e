// split_noalloc.hip -- the device form of the evaluation with its scratch in
// a file-scope device array instead of a caller workspace, for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// The array holds the same workspace split_eval_device carves from the
// caller's buffer (per-tour tables, partial-sum slots, the fallback list and
// value history); the tour-ordered demand copy is never used here, so the
// call always takes the path that stages tiles in LDS.  Every device the
// library runs on holds its own copy of the array until the process ends;
// its address is looked up once per device with that device current, and
// that address (never the array's name) is what host code hands the kernels.
// The kernels clear what must start at zero themselves (the prep kernel
// resets the slots and counters), so the call issues no memset.  Calls that
// overlap on one device share the array and race.

#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>

#include "split_check.h"
#include "split_eval.h"
#include "split_internal.h"

namespace {

constexpr size_t kScratchBytes = SPLIT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up once per
// device, with that device current).
int scratch_ptr(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return splitk::set_error(SPLIT_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return splitk::set_error(SPLIT_EDEVICE, "device %d outside the supported range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return splitk::set_error(SPLIT_EDEVICE, "scratch address: %s", hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SPLIT_OK;
}

} // namespace

extern "C" size_t split_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int split_eval_device_noalloc(const int32_t *d_tours, const int32_t *d_lens,
                                         int32_t num_tours, int32_t max_len,
                                         const int32_t *d_dist, int32_t N,
                                         const int16_t *d_demands, int64_t S, int32_t Q,
                                         int32_t *d_costs, int64_t *d_sums, double *d_means,
                                         split_stream_t stream)
{
    splitk::clear_error();
    int rc = splitk::check_scalars(num_tours, N, S, Q, max_len);
    if (rc)
        return rc;
    if (!d_tours || !d_lens || !d_dist || !d_demands || !d_costs || !d_sums || !d_means)
        return splitk::set_error(SPLIT_EINVAL, "null pointer argument");
    if (reinterpret_cast<uintptr_t>(d_demands) % 16)
        return splitk::set_error(SPLIT_EINVAL, "demands must be 16-byte aligned");
    const size_t need = splitk::workspace_bytes(num_tours, max_len, N, S, false);
    if (need > kScratchBytes)
        return splitk::set_error(SPLIT_EINVAL,
                                 "the call needs %zu bytes of scratch, the fixed array holds %zu "
                                 "(fewer tours, shorter tours or fewer scenarios per call)",
                                 need, kScratchBytes);
    void *ws_base = nullptr;
    rc = scratch_ptr(&ws_base);
    if (rc)
        return rc;
    bool ordered = false;
    splitk::Schedule sched = splitk::choose_schedule(num_tours, max_len, N, S, Q, &ordered);
    sched.path = 1; // tiles staged in LDS: no tour-ordered copy
    const splitk::Workspace ws =
        splitk::carve_workspace(ws_base, num_tours, max_len, N, S, false);
    const hipError_t e = splitk::launch_eval(d_tours, d_lens, num_tours, max_len, d_dist, N,
                                             d_demands, S, Q, d_costs, d_sums, d_means, ws,
                                             static_cast<hipStream_t>(stream), sched);
    if (e != hipSuccess)
        return splitk::set_error(SPLIT_EDEVICE, "launch: %s", hipGetErrorString(e));
    return SPLIT_OK;
}
