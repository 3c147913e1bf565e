// Host-only sanitizer driver for the library's argument checks (built with
// g++ -fsanitize=address,undefined by tests/test_sanitize.py; no device code).
// Every tour id is checked before it indexes the cost matrix, so the bad
// inputs below must be rejected without an out-of-bounds read.
#include <stdio.h>
#include <string.h>

#include <vector>

#include "split_check.h"
#include "split_eval.h"

extern "C" const char *split_last_error(void);

static int failures = 0;

static void expect(bool ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAIL: %s (last error: %s)\n", what, split_last_error());
        ++failures;
    }
}

int main()
{
    const int N = 20;
    const int N1 = N + 1;
    // the cost matrix sits in its own heap block, so a read past it is caught
    std::vector<int32_t> dist((size_t)N1 * N1);
    for (int a = 0; a <= N; ++a)
        for (int b = 0; b <= N; ++b)
            dist[(size_t)a * N1 + b] = a == b ? 0 : 10 + (a * 7 + b * 3) % 50;
    std::vector<int32_t> tour(N);
    for (int k = 0; k < N; ++k)
        tour[k] = k + 1;
    int32_t lens[2] = {N, 0};
    int32_t max_len = -1;
    int64_t total = -1;
    expect(splitk::check_tours_host(tour.data(), lens, 2, dist.data(), N, &max_len, &total) ==
               SPLIT_OK && max_len == N && total == N,
           "a valid tour and an empty tour pass");
    const int32_t bad_ids[] = {0, N + 1, 99, 1 << 30, -(1 << 30), -1, 2147483647};
    for (int pos : {0, 1, 7, N - 2, N - 1}) {
        for (int32_t id : bad_ids) {
            std::vector<int32_t> t = tour;
            t[pos] = id;
            const int rc = splitk::check_tours_host(t.data(), lens, 1, dist.data(), N, &max_len,
                                                    &total);
            expect(rc == SPLIT_EINVAL && strstr(split_last_error(), "outside [1") != nullptr,
                   "an id outside [1, N] at any position is rejected");
        }
    }
    {
        std::vector<int32_t> d = dist;
        d[(size_t)tour[3] * N1 + tour[4]] = -5;
        expect(splitk::check_tours_host(tour.data(), lens, 1, d.data(), N, &max_len, &total) ==
                   SPLIT_EINVAL,
               "a negative leg is rejected");
        d = dist;
        d[(size_t)tour[5] * N1 + 0] = SPLIT_MAX_COST + 1;
        expect(splitk::check_tours_host(tour.data(), lens, 1, d.data(), N, &max_len, &total) ==
                   SPLIT_EINVAL,
               "a leg above the largest cost is rejected");
        for (auto &v : d)
            v = v ? (1 << 24) : 0;
        expect(splitk::check_tours_host(tour.data(), lens, 1, d.data(), N, &max_len, &total) ==
                       SPLIT_EINVAL &&
                   strstr(split_last_error(), "guard") != nullptr,
               "the exactness guard is enforced");
    }
    int32_t bad_len[1] = {70000};
    expect(splitk::check_tours_host(tour.data(), bad_len, 1, dist.data(), N, &max_len, &total) ==
               SPLIT_EINVAL,
           "a length past the limit is rejected before any id is read");
    expect(splitk::check_scalars(0, N, 10, 3, 5) == SPLIT_EINVAL, "num_tours >= 1");
    expect(splitk::check_scalars(1, 0, 10, 3, 5) == SPLIT_EINVAL, "N >= 1");
    expect(splitk::check_scalars(1, N, 0, 3, 5) == SPLIT_EINVAL, "S >= 1");
    expect(splitk::check_scalars(1, N, 10, -1, 5) == SPLIT_EINVAL, "Q >= 0");
    expect(splitk::check_scalars(1, N, 10, 3, 70000) == SPLIT_EINVAL, "max_len bound");
    expect(splitk::check_scalars(1 << 20, N, (int64_t)1 << 40, 3, 5) == SPLIT_EINVAL,
           "unit count bound");
    expect(splitk::check_scalars(4, N, 1000, 3, 5) == SPLIT_OK, "valid scalars pass");
    // a long error text is truncated, not overrun
    std::vector<char> longfmt(2000, 'x');
    longfmt.back() = 0;
    splitk::set_error(SPLIT_EINVAL, "%s", longfmt.data());
    expect(strlen(split_last_error()) < 512, "error text is bounded");
    splitk::clear_error();
    expect(split_last_error()[0] == 0, "error text clears");
    if (failures == 0)
        printf("check driver: all expectations met\n");
    return failures == 0 ? 0 : 1;
}
