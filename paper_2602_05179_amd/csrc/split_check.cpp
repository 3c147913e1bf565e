// split_check.cpp -- host-side argument checks and error text of the C ABI
// (no device code; see split_check.h).

#include "split_check.h"

#include <stdio.h>

#include "split_eval.h"

namespace {

thread_local char g_err[512] = "";

constexpr int32_t kMaxLen = 65535; // longest tour the library accepts
constexpr int64_t kTile = 64;      // scenarios per unit of work

} // namespace

namespace splitk {

int vset_error(int code, const char *fmt, va_list ap)
{
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    return code;
}

int set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vset_error(code, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

int check_scalars(int32_t num_tours, int32_t N, int64_t S, int32_t Q, int32_t max_len)
{
    if (num_tours < 1)
        return set_error(SPLIT_EINVAL, "num_tours must be >= 1 (got %d)", num_tours);
    if (N < 1)
        return set_error(SPLIT_EINVAL, "N must be >= 1 (got %d)", N);
    if (S < 1)
        return set_error(SPLIT_EINVAL, "S must be >= 1 (got %lld)", (long long)S);
    if (Q < 0)
        return set_error(SPLIT_EINVAL, "Q must be >= 0 (got %d)", Q);
    if (max_len < 0 || max_len > kMaxLen)
        return set_error(SPLIT_EINVAL, "tour length must be in [0, %d] (got %d)", kMaxLen,
                         max_len);
    const int64_t tiles = (S + kTile - 1) / kTile;
    if ((int64_t)num_tours * tiles > (int64_t)INT32_MAX)
        return set_error(SPLIT_EINVAL, "num_tours * ceil(S/64) exceeds 2^31-1");
    return SPLIT_OK;
}

int check_tours_host(const int32_t *tours, const int32_t *lens, int32_t T, const int32_t *dist,
                     int32_t N, int32_t *max_len_out, int64_t *total_out)
{
    const int64_t N1 = (int64_t)N + 1;
    int64_t off = 0;
    int32_t max_len = 0;
    for (int32_t t = 0; t < T; ++t) {
        const int32_t n = lens[t];
        if (n < 0 || n > kMaxLen)
            return set_error(SPLIT_EINVAL, "lens[%d] = %d outside [0, %d]", t, n, kMaxLen);
        int64_t maxc = 0;
        for (int32_t k = 0; k < n; ++k) {
            const int32_t c = tours[off + k];
            if (c < 1 || c > N)
                return set_error(SPLIT_EINVAL,
                                 "tour %d position %d: customer id %d outside [1, %d]", t, k + 1,
                                 c, N);
            // the next id is checked before it indexes dist
            const int32_t cn = k + 1 < n ? tours[off + k + 1] : 0;
            if (k + 1 < n && (cn < 1 || cn > N))
                return set_error(SPLIT_EINVAL,
                                 "tour %d position %d: customer id %d outside [1, %d]", t, k + 2,
                                 cn, N);
            const int32_t legs[3] = {dist[c], dist[c * N1], k + 1 < n ? dist[c * N1 + cn] : 0};
            for (int32_t v : legs) {
                if (v < 0 || v > SPLIT_MAX_COST)
                    return set_error(SPLIT_EINVAL, "tour %d: travel cost %d outside [0, %d]", t,
                                     v, SPLIT_MAX_COST);
                if (v > maxc)
                    maxc = v;
            }
        }
        if (3 * (int64_t)n * maxc >= (int64_t)1 << 29)
            return set_error(SPLIT_EINVAL,
                             "tour %d: 3 * n * max cost = %lld >= 2^29 (int32 exactness guard)",
                             t, (long long)(3 * (int64_t)n * maxc));
        if (n > max_len)
            max_len = n;
        off += n;
    }
    *max_len_out = max_len;
    *total_out = off;
    return SPLIT_OK;
}

} // namespace splitk

extern "C" const char *split_last_error(void) { return g_err; }
