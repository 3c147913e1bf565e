// split_variant.h -- host-side entry of the split-variant kernels (soft
// capacity, fleet bound); not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace splitk {

// Workspace of a variant call: the evaluator's one-tour workspace (with the
// tour-ordered copy when that path is taken), two
// position-major potential buffers [n][S] when K > 0, and the exact
// fallback's two value arrays per block.
size_t variant_workspace_bytes(int32_t n, int32_t N, int64_t S, int32_t K);

// Whether a call streams the tour-ordered copy of the demands (path
// override, else by the demand bytes per wave of the LDS tile); the
// workspace holds the copy then.
bool variants_ordered(int32_t n, int32_t N, int32_t K);
void set_variant_path(int path); // 0 automatic, 1 LDS tile, 2 tour-ordered copy

// Register ring length used for this capacity (32, or 64 above Q = 200).
int variant_ring(int32_t Q);

// Enqueues prep, the variant tile kernel and the exact fallback (whose last
// block writes *status: 0, or the bit set of validation failures).
hipError_t launch_variant(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                          const int16_t *demands, int64_t S, int32_t Q, int32_t beta, int32_t K,
                          int32_t *costs, int32_t *status, void *workspace, hipStream_t stream);

} // namespace splitk
