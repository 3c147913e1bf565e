// split_small.h -- the one-launch form of the plain split for small
// problems (split_small.hip); not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "split_internal.h"

namespace splitk {

// Serial recursion steps one wave may take (tiles per wave x tour length)
// before the general path, which spreads the tiles over the whole chip,
// is the faster one.
constexpr int64_t kSmallMaxSteps = 256;

// Largest customer pool: eight staged 64 x N byte tiles (128 KB at N = 256)
// in one workgroup's LDS.  Larger pools take the tour-ordered path anyway.
constexpr int32_t kSmallMaxN = 256;

// whether a call takes the one-launch form: one tour, a short serial
// chain per wave, a pool of at most kSmallMaxN customers, the path left to the automatic choice (a forced path takes
// the general kernels)
bool small_path_fits(int32_t num_tours, int32_t max_len, int32_t N, int64_t S,
                     const Schedule &s, bool ordered);

// one-time set-up of the one-launch kernels (their LDS limit), done by the
// first launch; a caller about to capture a graph calls it first, so that
// no such set-up falls inside the capture
hipError_t small_prepare();

// tables, recursion, exact fallback and the fold in one launch; the same
// workspace layout, costs, sums and means as launch_eval for one tour
hipError_t launch_small(const int32_t *tours, const int32_t *lens, int32_t max_len,
                        const int32_t *dist, int32_t N, const int16_t *demands, int64_t S,
                        int32_t Q, int32_t *costs, int64_t *sums, double *means,
                        const Workspace &ws, hipStream_t stream, const Schedule &s);

} // namespace splitk
