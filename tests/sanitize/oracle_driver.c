/* Host-only sanitizer driver for the CPU oracle (built with gcc
 * -fsanitize=address,undefined by tests/test_sanitize.py): every entry point
 * on small random instances, ragged and empty tours, infeasible scenarios and
 * the break / no-break walks; results are cross-checked where two entry
 * points compute the same thing. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_split_eval(const int32_t *tours, const int32_t *lens, int32_t num_tours, const int32_t *dist,
                      int32_t N, const int16_t *demands, int64_t S, int32_t Q, int32_t *costs,
                      int64_t *sums, double *means, int64_t *cells, int use_break, int nthreads);
int oracle_split_values(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                        const int64_t *qvis, int64_t Q, int use_break, int64_t *V_out, int64_t *cells_out);
int oracle_split_routes(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                        const int16_t *demands, int64_t S, int32_t Q, int32_t *costs,
                        uint16_t *pred, uint16_t *cuts, int32_t *nroutes, int nthreads);
int oracle_split_variant(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                         const int16_t *demands, int64_t S, int32_t Q, int32_t beta, int32_t K,
                         int64_t *costs, int nthreads);

static uint64_t rs = 88172645463325252ull;
static int rnd(int lo, int hi) /* xorshift64, inclusive range */
{
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return lo + (int)(rs % (uint64_t)(hi - lo + 1));
}

static int failures = 0;
#define EXPECT(c, what)                                                                            \
    do {                                                                                           \
        if (!(c)) {                                                                                \
            fprintf(stderr, "FAIL: %s\n", what);                                                   \
            ++failures;                                                                            \
        }                                                                                          \
    } while (0)

int main(void)
{
    for (int trial = 0; trial < 40; ++trial) {
        const int N = rnd(1, 30), S = rnd(1, 70), T = rnd(1, 4), Q = rnd(0, 40);
        const int N1 = N + 1;
        int32_t *dist = malloc(sizeof(int32_t) * N1 * N1);
        for (int a = 0; a < N1 * N1; ++a)
            dist[a] = rnd(0, 100);
        int16_t *dem = malloc(sizeof(int16_t) * S * N);
        for (int a = 0; a < S * N; ++a)
            dem[a] = (int16_t)rnd(0, Q + 3);
        int32_t lens[4];
        int total = 0;
        for (int t = 0; t < T; ++t) {
            lens[t] = rnd(0, 2 * N);
            total += lens[t];
        }
        int32_t *tours = malloc(sizeof(int32_t) * (total ? total : 1));
        for (int k = 0; k < total; ++k)
            tours[k] = rnd(1, N);
        int32_t *c1 = malloc(sizeof(int32_t) * T * S), *c2 = malloc(sizeof(int32_t) * T * S);
        int64_t sums[4], sums2[4], cells[4];
        double means[4];
        EXPECT(oracle_split_eval(tours, lens, T, dist, N, dem, S, Q, c1, sums, means, cells, 1, 2) == 0,
               "eval with break");
        EXPECT(oracle_split_eval(tours, lens, T, dist, N, dem, S, Q, c2, sums2, means, NULL, 0, 1) == 0,
               "eval without break");
        for (int a = 0; a < T * S; ++a)
            EXPECT(c1[a] == c2[a], "break and full walk agree");
        int off = 0;
        for (int t = 0; t < T; ++t) {
            const int n = lens[t];
            const int32_t *tour = tours + off;
            int32_t *rc = malloc(sizeof(int32_t) * S), *nr = malloc(sizeof(int32_t) * S);
            uint16_t *pred = malloc(sizeof(uint16_t) * (n ? n : 1) * S);
            uint16_t *cuts = malloc(sizeof(uint16_t) * (n ? n : 1) * S);
            EXPECT(oracle_split_routes(tour, n, dist, N, dem, S, Q, rc, pred, cuts, nr, 2) == 0, "routes");
            int64_t *vc = malloc(sizeof(int64_t) * S);
            EXPECT(oracle_split_variant(tour, n, dist, N, dem, S, Q, -1, 0, vc, 2) == 0, "variant");
            int64_t *qv = malloc(sizeof(int64_t) * (n ? n : 1));
            int64_t *V = malloc(sizeof(int64_t) * (n + 1));
            for (int s = 0; s < S; ++s) {
                EXPECT(rc[s] == c1[t * S + s], "routes cost = eval cost");
                EXPECT((vc[s] == INT64_MAX ? INT32_MAX : vc[s]) == c1[t * S + s],
                       "hard unlimited variant = eval cost");
                for (int k = 0; k < n; ++k)
                    qv[k] = dem[(int64_t)s * N + tour[k] - 1];
                int64_t cc = 0;
                EXPECT(oracle_split_values(tour, n, dist, N, qv, Q, 1, V, &cc) == 0, "values");
                EXPECT((V[n] == INT64_MAX ? INT32_MAX : V[n]) == c1[t * S + s], "values(n) = eval cost");
            }
            const int beta = rnd(0, 9), K = rnd(0, 4);
            EXPECT(oracle_split_variant(tour, n, dist, N, dem, S, Q, beta, K, vc, 1) == 0, "soft variant");
            free(rc); free(nr); free(pred); free(cuts); free(vc); free(qv); free(V);
            off += n;
        }
        free(dist); free(dem); free(tours); free(c1); free(c2);
    }
    if (failures == 0)
        printf("oracle driver: all expectations met\n");
    return failures == 0 ? 0 : 1;
}
