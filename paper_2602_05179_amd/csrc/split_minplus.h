// split_minplus.h -- host-side entry of the min-plus kernels (not part of the
// public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace splitk {

constexpr int kMinplusMaxStates = 4096; // states per stage (LDS: 2 * m int32 per wave)
constexpr int kOuMaxStates = 32;        // inventory levels of the fused order-up-to DP (U <= 31)

hipError_t launch_minplus_forward(const int32_t *A, int32_t shared, int32_t T, int32_t m,
                                  int64_t B, const int32_t *J0, int32_t *JT, int32_t *arg,
                                  hipStream_t stream);
hipError_t launch_minplus_backtrack(const int32_t *JT, const int32_t *arg, int32_t T, int32_t m,
                                    int64_t B, int32_t *path, hipStream_t stream);
hipError_t launch_ou_transitions(int32_t U, int32_t T, int64_t B, int32_t R,
                                 const int32_t *demand, const int32_t *opt_cost,
                                 const int32_t *opt_cap, const int32_t *h, int32_t u, int32_t rho,
                                 int32_t *A, hipStream_t stream);
hipError_t launch_ou_dp(int32_t U, int32_t T, int64_t B, int32_t R, const int32_t *demand,
                        const int32_t *opt_cost, const int32_t *opt_cap, const int32_t *h,
                        int32_t u, int32_t rho, const int32_t *J0, int32_t *JT, int32_t *arg,
                        int32_t *status, hipStream_t stream);

} // namespace splitk
