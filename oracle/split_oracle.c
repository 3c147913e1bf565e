/*
 * split_oracle.c -- CPU oracle for the scenario-batched split recursion.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or helper with the HIP
 * library.
 *
 * What it computes (paper Sec. 2.3, "Forward DP recursion and matrix form",
 * and the worked 3-customer example of App. A):
 *
 *   For a giant tour sigma = (sigma_1..sigma_n) and one demand scenario w,
 *     W(p,i)  = c[0][sigma_{p+1}] + sum_{k=p+1}^{i-1} c[sigma_k][sigma_{k+1}]
 *               + c[sigma_i][depot]                     (route p+1..i)
 *     A(p,i)  = W(p,i) if p < i and sum_{k=p+1}^{i} q_w(sigma_k) <= Q,
 *               +inf otherwise                          (capacity mask)
 *     J(0)    = 0,  J(i) = min_{p<i} J(p) + A(p,i),  i = 1..n.
 *   The second-stage cost of scenario w is J(n); the sample-average
 *   estimate is (1/|Omega|) sum_w J_w(n) with equal weights (App. A,
 *   extensive-form objective).
 *
 * Readings where the paper is silent (each one is listed in the design
 * notes): the destination depot n+1 is the depot, node 0; demands are
 * indexed by customer id; load equal to Q is feasible (the worked example
 * accepts a route of load exactly Q); the fleet is unlimited; a scenario in
 * which no split exists (some customer's demand exceeds Q) has cost +inf,
 * reported as INT32_MAX per scenario, INT64_MAX as the tour's sum and +inf
 * as its mean; an empty tour costs 0.
 *
 * This is the plain O(n^2) Bellman loop: for every i it walks the
 * predecessors p = i-1, i-2, ..., 0 while accumulating the route's load and
 * its inner arc length.  Because demands are non-negative the load only
 * grows as p decreases, so once it exceeds Q every smaller p is infeasible
 * too; `use_break` stops the walk there (an exact shortcut), and with
 * use_break = 0 the walk visits every p and masks the infeasible ones.  All
 * arithmetic is int64, so there is no overflow question here at all.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_INF INT64_MAX

/* One scenario.  q[k] = demand of tour position k (1-based, q[0] unused),
 * V must hold n+1 entries.  Returns J(n) or OR_INF; adds the number of
 * capacity-feasible (p,i) relaxations to *cells. */
static int64_t split_one(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N1,
                         const int64_t *q, int64_t Q, int use_break, int64_t *V, int64_t *cells)
{
    V[0] = 0;
    for (int32_t i = 1; i <= n; ++i) {
        const int32_t last = tour[i - 1];                 /* sigma_i */
        const int64_t back = dist[(int64_t)last * N1 + 0];  /* c[sigma_i][depot] */
        int64_t best = OR_INF;
        int64_t load = 0;
        int64_t inner = 0; /* sum_{k=p+1}^{i-1} c[sigma_k][sigma_{k+1}] */
        for (int32_t p = i - 1; p >= 0; --p) {
            const int32_t first = tour[p];                /* sigma_{p+1} */
            load += q[p + 1];
            if (p + 1 <= i - 1) {
                const int32_t nxt = tour[p + 1];          /* sigma_{p+2} */
                inner += dist[(int64_t)first * N1 + nxt];
            }
            if (load > Q) {
                if (use_break)
                    break;
                continue;
            }
            *cells += 1;
            const int64_t w = dist[first] /* c[0][sigma_{p+1}] */ + inner + back;
            if (V[p] != OR_INF && V[p] + w < best)
                best = V[p] + w;
        }
        V[i] = best;
    }
    return V[n];
}

typedef struct {
    const int32_t *tour;
    int32_t n;
    const int32_t *dist;
    int32_t N;
    const int16_t *demands;
    int64_t s_begin, s_end;
    int64_t Q;
    int use_break;
    int32_t *costs;     /* indexed by scenario */
    int64_t sum;        /* exact sum of finite costs */
    int64_t n_inf;
    int64_t cells;
    int status;
} job_t;

static void *run_job(void *arg)
{
    job_t *jb = (job_t *)arg;
    const int32_t N1 = jb->N + 1;
    int64_t *V = (int64_t *)malloc(sizeof(int64_t) * ((size_t)jb->n + 1));
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * ((size_t)jb->n + 1));
    if (!V || !q) {
        jb->status = -2;
        free(V);
        free(q);
        return NULL;
    }
    for (int64_t s = jb->s_begin; s < jb->s_end; ++s) {
        const int16_t *row = jb->demands + s * (int64_t)jb->N;
        q[0] = 0;
        for (int32_t k = 1; k <= jb->n; ++k)
            q[k] = row[jb->tour[k - 1] - 1];
        const int64_t v = split_one(jb->tour, jb->n, jb->dist, N1, q, jb->Q, jb->use_break, V,
                                    &jb->cells);
        if (v == OR_INF) {
            jb->costs[s] = INT32_MAX;
            jb->n_inf += 1;
        } else {
            jb->costs[s] = (int32_t)v;
            jb->sum += v;
        }
    }
    free(V);
    free(q);
    return NULL;
}

/* Validate the call the same way the library's contract states. */
static int check_args(const int32_t *tours, const int32_t *lens, int32_t num_tours, const int32_t *dist,
                      int32_t N, const int16_t *demands, int64_t S, int32_t Q)
{
    if (!tours || !lens || !dist || !demands || num_tours < 1 || N < 1 || S < 1 || Q < 0)
        return -1;
    int64_t off = 0;
    for (int32_t t = 0; t < num_tours; ++t) {
        if (lens[t] < 0)
            return -1;
        for (int32_t k = 0; k < lens[t]; ++k)
            if (tours[off + k] < 1 || tours[off + k] > N)
                return -1;
        off += lens[t];
    }
    return 0;
}

/*
 * Evaluate every tour on every scenario.
 *   costs  [num_tours * S] int32 : J_w(n_t), INT32_MAX where no split exists
 *   sums   [num_tours]     int64 : exact sum over scenarios, INT64_MAX if any +inf
 *   means  [num_tours]     double: sum / S (one IEEE division), +inf if any +inf
 *   cells  [num_tours]     int64 : number of capacity-feasible relaxations
 * nthreads >= 1 splits each tour's scenarios into contiguous blocks.
 * Returns 0, -1 on invalid arguments, -2 on allocation failure.
 */
int oracle_split_eval(const int32_t *tours, const int32_t *lens, int32_t num_tours, const int32_t *dist,
                      int32_t N, const int16_t *demands, int64_t S, int32_t Q, int32_t *costs,
                      int64_t *sums, double *means, int64_t *cells, int use_break, int nthreads)
{
    if (check_args(tours, lens, num_tours, dist, N, demands, S, Q) != 0)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    if ((int64_t)nthreads > S)
        nthreads = (int)S;
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return -2;
    }
    int rc = 0;
    int64_t off = 0;
    for (int32_t t = 0; t < num_tours && rc == 0; ++t) {
        for (int k = 0; k < nthreads; ++k) {
            job_t *jb = &jobs[k];
            memset(jb, 0, sizeof(*jb));
            jb->tour = tours + off;
            jb->n = lens[t];
            jb->dist = dist;
            jb->N = N;
            jb->demands = demands;
            jb->s_begin = S * k / nthreads;
            jb->s_end = S * (k + 1) / nthreads;
            jb->Q = Q;
            jb->use_break = use_break;
            jb->costs = costs + (int64_t)t * S;
        }
        if (nthreads == 1) {
            run_job(&jobs[0]);
        } else {
            for (int k = 0; k < nthreads; ++k)
                pthread_create(&th[k], NULL, run_job, &jobs[k]);
            for (int k = 0; k < nthreads; ++k)
                pthread_join(th[k], NULL);
        }
        int64_t sum = 0, n_inf = 0, c = 0;
        for (int k = 0; k < nthreads; ++k) {
            if (jobs[k].status)
                rc = jobs[k].status;
            sum += jobs[k].sum;
            n_inf += jobs[k].n_inf;
            c += jobs[k].cells;
        }
        if (sums)
            sums[t] = n_inf ? INT64_MAX : sum;
        if (means)
            means[t] = n_inf ? INFINITY : (double)sum / (double)S;
        if (cells)
            cells[t] = c;
        off += lens[t];
    }
    free(jobs);
    free(th);
    return rc;
}

/*
 * Full value vector J(0..n) of one scenario given demands in visiting
 * order (qvis[k-1] = demand of sigma_k).  Entries with no split are
 * INT64_MAX.  Used by the pin tests on tiny worked examples.
 */
int oracle_split_values(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                        const int64_t *qvis, int64_t Q, int use_break, int64_t *V_out, int64_t *cells_out)
{
    if (!tour || !dist || !qvis || !V_out || n < 0 || N < 1 || Q < 0)
        return -1;
    for (int32_t k = 0; k < n; ++k)
        if (tour[k] < 1 || tour[k] > N || qvis[k] < 0)
            return -1;
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!q)
        return -2;
    q[0] = 0;
    for (int32_t k = 1; k <= n; ++k)
        q[k] = qvis[k - 1];
    int64_t c = 0;
    split_one(tour, n, dist, N + 1, q, Q, use_break, V_out, &c);
    if (cells_out)
        *cells_out = c;
    free(q);
    return 0;
}

/*
 * Route recovery.  The giant tour is cut into routes by the split (App. A:
 * routes are recovered from the giant tour by the split operator), and a
 * DP that records each minimiser is backtracked to recover the decisions
 * (App. B, batched DP with backtracking).  Readings where the paper is
 * silent: pred(i) is the SMALLEST predecessor p attaining J(i) =
 * J(p) + A(p,i) (ties broken towards longer last routes), 0xFFFF when
 * J(i) = +inf; the cut points are i_k = n, i_{k-1} = pred(i_k), ..., down
 * to 0, reported in increasing order (the route ends), so route r covers
 * positions i_{r-1}+1 .. i_r with i_0 = 0.
 */
#define OR_NO_PRED 0xFFFFu

static int64_t split_one_pred(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N1,
                              const int64_t *q, int64_t Q, int64_t *V, uint16_t *pred)
{
    V[0] = 0;
    for (int32_t i = 1; i <= n; ++i) {
        const int32_t last = tour[i - 1];
        const int64_t back = dist[(int64_t)last * N1 + 0];
        int64_t best = OR_INF;
        int32_t arg = -1;
        int64_t load = 0;
        int64_t inner = 0;
        for (int32_t p = i - 1; p >= 0; --p) { /* p decreasing: "<=" keeps the smallest */
            const int32_t first = tour[p];
            load += q[p + 1];
            if (p + 1 <= i - 1)
                inner += dist[(int64_t)first * N1 + tour[p + 1]];
            if (load > Q)
                break;
            const int64_t w = dist[first] + inner + back;
            if (V[p] != OR_INF && V[p] + w <= best) {
                best = V[p] + w;
                arg = p;
            }
        }
        V[i] = best;
        pred[i - 1] = arg < 0 ? (uint16_t)OR_NO_PRED : (uint16_t)arg;
    }
    return V[n];
}

typedef struct {
    const int32_t *tour;
    int32_t n;
    const int32_t *dist;
    int32_t N;
    const int16_t *demands;
    int64_t s_begin, s_end;
    int64_t Q;
    int32_t *costs;
    uint16_t *pred;
    uint16_t *cuts;
    int32_t *nroutes;
    int status;
} routes_job_t;

static void *run_routes_job(void *arg)
{
    routes_job_t *jb = (routes_job_t *)arg;
    const int32_t n = jb->n;
    int64_t *V = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    uint16_t *pr = (uint16_t *)malloc(sizeof(uint16_t) * ((size_t)n + 1));
    if (!V || !q || !pr) {
        jb->status = -2;
        free(V);
        free(q);
        free(pr);
        return NULL;
    }
    for (int64_t s = jb->s_begin; s < jb->s_end; ++s) {
        const int16_t *row = jb->demands + s * (int64_t)jb->N;
        q[0] = 0;
        for (int32_t k = 1; k <= n; ++k)
            q[k] = row[jb->tour[k - 1] - 1];
        const int64_t v = split_one_pred(jb->tour, n, jb->dist, jb->N + 1, q, jb->Q, V, pr);
        jb->costs[s] = v == OR_INF ? INT32_MAX : (int32_t)v;
        if (jb->pred)
            memcpy(jb->pred + s * (int64_t)n, pr, sizeof(uint16_t) * (size_t)n);
        uint16_t *cut = jb->cuts ? jb->cuts + s * (int64_t)n : NULL;
        if (cut)
            memset(cut, 0, sizeof(uint16_t) * (size_t)n);
        int32_t k = 0;
        if (v != OR_INF) {
            for (int32_t i = n; i > 0; i = pr[i - 1])
                ++k;
            int32_t r = k;
            for (int32_t i = n; i > 0; i = pr[i - 1])
                if (cut)
                    cut[--r] = (uint16_t)i;
        }
        jb->nroutes[s] = k;
    }
    free(V);
    free(q);
    free(pr);
    return NULL;
}

/*
 * Route recovery for one tour over every scenario: costs[s] = J_s(n)
 * (INT32_MAX if no split exists), pred[s*n + i-1] = pred_s(i) (may be
 * NULL), cuts[s*n + r-1] = end position of route r (r = 1..nroutes[s],
 * zeros after; may be NULL), nroutes[s] = number of routes (0 for an
 * infeasible scenario or an empty tour).  n must fit 16-bit positions.
 */
int oracle_split_routes(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                        const int16_t *demands, int64_t S, int32_t Q, int32_t *costs,
                        uint16_t *pred, uint16_t *cuts, int32_t *nroutes, int nthreads)
{
    int32_t lens = n;
    if (check_args(tour, &lens, 1, dist, N, demands, S, Q) != 0 || !costs || !nroutes ||
        n > 65535)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 64)
        nthreads = 64;
    if ((int64_t)nthreads > S)
        nthreads = (int)S;
    routes_job_t jobs[64];
    pthread_t th[64];
    for (int w = 0; w < nthreads; ++w) {
        routes_job_t *jb = &jobs[w];
        jb->tour = tour;
        jb->n = n;
        jb->dist = dist;
        jb->N = N;
        jb->demands = demands;
        jb->s_begin = S * w / nthreads;
        jb->s_end = S * (w + 1) / nthreads;
        jb->Q = Q;
        jb->costs = costs;
        jb->pred = pred;
        jb->cuts = cuts;
        jb->nroutes = nroutes;
        jb->status = 0;
    }
    int created[64] = {0};
    for (int w = 1; w < nthreads; ++w)
        created[w] = pthread_create(&th[w], NULL, run_routes_job, &jobs[w]) == 0;
    run_routes_job(&jobs[0]);
    int rc = jobs[0].status;
    for (int w = 1; w < nthreads; ++w) {
        if (created[w])
            pthread_join(th[w], NULL);
        else
            run_routes_job(&jobs[w]); /* no thread: run it here */
        if (jobs[w].status && !rc)
            rc = jobs[w].status;
    }
    return rc;
}

/*
 * Split variants from the extensive form's objective and constraints
 * (App. A): every route pays its overload at rate beta, i.e. the route
 * p+1..i costs
 *     W(p,i) + beta * max(0, load(p+1..i) - Q)        (soft capacity)
 * instead of being excluded when its load exceeds Q, and at most K routes
 * may be used (the fleet-size bound).  With J_k(i) the cheapest split of
 * positions 1..i into exactly k routes,
 *     J_0(0) = 0,  J_0(i) = +inf for i > 0,
 *     J_k(i) = min_{p<i} J_{k-1}(p) + cost(p,i),
 * and the scenario's cost is min_{k<=K} J_k(n).  K = 0 means an unlimited
 * fleet: J(i) = min_{p<i} J(p) + cost(p,i) as in the plain recursion.
 * beta < 0 keeps the hard capacity (overloaded routes excluded, as in the
 * plain recursion), so (beta < 0, K = 0) is the plain split.  Readings: the
 * penalty is linear in the overload of each route (one l_k per vehicle);
 * an empty tour costs 0 for every K.
 *
 * costs[s] (int64) = the scenario's cost, INT64_MAX if no split exists.
 */
static int64_t variant_cost(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N1,
                            const int64_t *q, int64_t Q, int64_t beta, int32_t K, int64_t *Va,
                            int64_t *Vb)
{
    if (n == 0)
        return 0;
    const int layered = K > 0;
    const int32_t layers = layered ? K : 1;
    int64_t *prev = Va, *cur = Vb;
    for (int32_t i = 0; i <= n; ++i)
        prev[i] = i == 0 ? 0 : OR_INF; /* J_0 */
    int64_t ans = OR_INF;
    for (int32_t k = 1; k <= layers; ++k) {
        /* unlimited fleet: one array, each J(i) built from J(p < i) of itself */
        int64_t *src = layered ? prev : cur;
        cur[0] = layered ? OR_INF : 0;
        for (int32_t i = 1; i <= n; ++i) {
            const int32_t last = tour[i - 1];
            const int64_t back = dist[(int64_t)last * N1 + 0];
            int64_t best = OR_INF, load = 0, inner = 0;
            for (int32_t p = i - 1; p >= 0; --p) {
                const int32_t first = tour[p];
                load += q[p + 1];
                if (p + 1 <= i - 1)
                    inner += dist[(int64_t)first * N1 + tour[p + 1]];
                if (beta < 0 && load > Q)
                    break; /* hard capacity: every smaller p overloads too */
                int64_t w = dist[first] + inner + back;
                if (beta >= 0 && load > Q)
                    w += beta * (load - Q);
                if (src[p] != OR_INF && src[p] + w < best)
                    best = src[p] + w;
            }
            cur[i] = best;
        }
        if (cur[n] < ans)
            ans = cur[n];
        int64_t *t = prev;
        prev = cur;
        cur = t;
    }
    return ans;
}

typedef struct {
    const int32_t *tour;
    int32_t n;
    const int32_t *dist;
    int32_t N;
    const int16_t *demands;
    int64_t s_begin, s_end;
    int64_t Q, beta;
    int32_t K;
    int64_t *costs;
    int status;
} variant_job_t;

static void *run_variant_job(void *arg)
{
    variant_job_t *jb = (variant_job_t *)arg;
    const int32_t n = jb->n;
    int64_t *Va = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t *Vb = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!Va || !Vb || !q) {
        jb->status = -2;
        free(Va);
        free(Vb);
        free(q);
        return NULL;
    }
    for (int64_t s = jb->s_begin; s < jb->s_end; ++s) {
        const int16_t *row = jb->demands + s * (int64_t)jb->N;
        q[0] = 0;
        for (int32_t k = 1; k <= n; ++k)
            q[k] = row[jb->tour[k - 1] - 1];
        jb->costs[s] = variant_cost(jb->tour, n, jb->dist, jb->N + 1, q, jb->Q, jb->beta, jb->K,
                                    Va, Vb);
    }
    free(Va);
    free(Vb);
    free(q);
    return NULL;
}

int oracle_split_variant(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                         const int16_t *demands, int64_t S, int32_t Q, int32_t beta, int32_t K,
                         int64_t *costs, int nthreads)
{
    int32_t lens = n;
    if (check_args(tour, &lens, 1, dist, N, demands, S, Q) != 0 || !costs || K < 0)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 64)
        nthreads = 64;
    if ((int64_t)nthreads > S)
        nthreads = (int)S;
    variant_job_t jobs[64];
    pthread_t th[64];
    for (int w = 0; w < nthreads; ++w) {
        variant_job_t *jb = &jobs[w];
        jb->tour = tour;
        jb->n = n;
        jb->dist = dist;
        jb->N = N;
        jb->demands = demands;
        jb->s_begin = S * w / nthreads;
        jb->s_end = S * (w + 1) / nthreads;
        jb->Q = Q;
        jb->beta = beta;
        jb->K = K;
        jb->costs = costs;
        jb->status = 0;
    }
    int created[64] = {0};
    for (int w = 1; w < nthreads; ++w)
        created[w] = pthread_create(&th[w], NULL, run_variant_job, &jobs[w]) == 0;
    run_variant_job(&jobs[0]);
    int rc = jobs[0].status;
    for (int w = 1; w < nthreads; ++w) {
        if (created[w])
            pthread_join(th[w], NULL);
        else
            run_variant_job(&jobs[w]);
        if (jobs[w].status && !rc)
            rc = jobs[w].status;
    }
    return rc;
}
