// split_check.h -- host-side argument checks and the thread-local error text
// of the C ABI.  Plain C++ (no HIP), so the checks also build into a host-only
// sanitizer binary.
#pragma once

#include <stdarg.h>
#include <stdint.h>

namespace splitk {

// Thread-local error text returned by split_last_error().
int set_error(int code, const char *fmt, ...);
int vset_error(int code, const char *fmt, va_list ap);
void clear_error();

// Checks that need only scalars (shared by every form).
int check_scalars(int32_t num_tours, int32_t N, int64_t S, int32_t Q, int32_t max_len);

// Host-side validation of tours and the cost legs they use (host form):
// every id in [1, N] before it indexes dist, every leg in [0, SPLIT_MAX_COST],
// and the exactness guard 3 * n * max leg < 2^29.  Outputs the longest tour
// and the total length.
int check_tours_host(const int32_t *tours, const int32_t *lens, int32_t T, const int32_t *dist,
                     int32_t N, int32_t *max_len_out, int64_t *total_out);

} // namespace splitk
