// split_values.h -- launcher of the full value table (split_values.hip);
// not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "split_internal.h"

namespace splitk {

// prep of the single tour into `ws` (carved for one tour of length n),
// then V[(j-1)*S + s] = V_s(j) for j = 1..n; *status = 1 when a negative
// demand was read (that scenario's entries are SPLIT_INF).
hipError_t launch_values(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                         const int16_t *demands, int64_t S, int32_t Q, int32_t *V,
                         int32_t *status, const Workspace &ws, hipStream_t stream);

} // namespace splitk
