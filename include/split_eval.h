/*
 * split_eval.h -- C ABI of the MI355X scenario-batched split evaluator.
 *
 * Operation (paper Sec. 2.3, "Forward DP recursion and matrix form"; the
 * sample-average objective of App. A):
 *
 *   For a giant tour sigma = (sigma_1..sigma_n) of customer ids, a travel
 *   cost matrix c (node 0 = depot, which is also the destination depot) and
 *   one demand scenario w, the route serving tour positions p+1..i costs
 *     W(p,i) = c[0][sigma_{p+1}] + sum_{k=p+1}^{i-1} c[sigma_k][sigma_{k+1}]
 *              + c[sigma_i][0]
 *   and is admissible when its load sum_{k=p+1}^{i} q_w(sigma_k) <= Q.
 *     V_w(0) = 0,   V_w(i) = min over admissible p < i of V_w(p) + W(p,i).
 *   The second-stage cost of scenario w is V_w(n); the tour's SAA estimate
 *   is the equal-weight mean of V_w(n) over all scenarios.
 *
 * Conventions (all integers little-endian, arrays row-major):
 *   - customers are 1..N, node 0 is the depot; fleet size is unlimited;
 *   - a route whose load equals Q is admissible;
 *   - a scenario with no admissible split (some demand > Q) costs SPLIT_INF;
 *     the tour's sum is then INT64_MAX and its mean +infinity;
 *   - an empty tour (n = 0) costs 0 in every scenario;
 *   - all tours of one call share the scenario set (common random numbers).
 *
 * Input limits (violations give SPLIT_EINVAL):
 *   N >= 1, S >= 1, num_tours >= 1, 0 <= lens[t] <= max_len, Q >= 0,
 *   tour ids in [1, N], every cost on a tour's route legs (depot legs and
 *   consecutive arcs) in [0, SPLIT_MAX_COST], and
 *   3 * n_t * (largest such cost) < 2^29 so that all int32 arithmetic is
 *   exact; demands in [0, 32767] (int16, negative values are rejected).
 *
 * Results are bit-exact: per-scenario costs are int32, the sum is an exact
 * int64, the mean is that int64 divided by S in one IEEE double division.
 */
#ifndef SPLIT_EVAL_H
#define SPLIT_EVAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPLIT_OK 0
#define SPLIT_EINVAL (-1)  /* bad argument; see the limits above */
#define SPLIT_ENOMEM (-2)  /* device allocation failed or over the memory budget */
#define SPLIT_EDEVICE (-3) /* HIP runtime error; text in split_last_error() */
#define SPLIT_EAGAIN (-4)  /* served form: result not ready yet */

#define SPLIT_INF INT32_MAX             /* per-scenario cost when no split exists */
#define SPLIT_SUM_INVALID INT64_MIN     /* device-form sum of a tour whose inputs were invalid */
#define SPLIT_MAX_COST (1 << 24)        /* largest admissible single travel cost */

/* Opaque handles. */
typedef struct split_plan split_plan;
typedef struct split_server split_server;
/* HIP stream handle (hipStream_t), passed as an opaque pointer. */
typedef void *split_stream_t;

/*
 * Text of the last error on the calling thread ("" if none).  The pointer
 * stays valid until the next library call on the same thread.
 */
const char *split_last_error(void);

/*
 * split_eval -- evaluate num_tours giant tours on S demand scenarios.
 * Every pointer is HOST memory; the call is synchronous and keeps no
 * pointer after it returns.  The caller owns all buffers.
 *
 *   tours   int32 [sum(lens)]   concatenated tours (customer ids 1..N)
 *   lens    int32 [num_tours]   tour lengths n_t >= 0
 *   dist    int32 [(N+1)*(N+1)] dist[a*(N+1)+b] = cost of arc a -> b
 *   demands int16 [S*N]         scenario-major: demands[s*N + (c-1)]
 *   Q       vehicle capacity
 *   costs   out int32 [num_tours*S]  costs[t*S + s] = V_s(n_t) or SPLIT_INF
 *   sums    out int64 [num_tours]    exact sums (INT64_MAX if any SPLIT_INF); may be NULL
 *   means   out double [num_tours]   sums/S (+inf if any SPLIT_INF); may be NULL
 *
 * Returns SPLIT_OK, or an error code with the outputs left untouched.
 */
int split_eval(const int32_t *tours, const int32_t *lens, int32_t num_tours, const int32_t *dist,
               int32_t N, const int16_t *demands, int64_t S, int32_t Q, int32_t *costs,
               int64_t *sums, double *means);

/*
 * Device-memory workspace needed by split_eval_device for these sizes under
 * the schedule the library would pick now (override, tuned entry or
 * default).  Ask again after tuning or changing the schedule.
 */
size_t split_workspace_bytes(int32_t num_tours, int32_t max_len, int32_t N, int64_t S, int32_t Q);

/*
 * split_eval_device -- same operation on DEVICE pointers, enqueued on
 * `stream`; returns once the work is enqueued (nothing is allocated, no
 * host synchronisation, no memset or copy: safe to capture in a HIP graph).
 *
 *   d_tours, d_lens, d_dist, d_demands : device inputs as in split_eval;
 *       d_demands must be 16-byte aligned.
 *   max_len   host-side upper bound on every lens[t] (sizes the workspace)
 *   d_costs, d_sums, d_means : device outputs as in split_eval (none NULL)
 *   d_workspace, ws_bytes : caller-owned device scratch of at least
 *       split_workspace_bytes(num_tours, max_len, N, S) bytes, 256-aligned.
 *
 * Host-checkable arguments (sizes, Q, alignment, workspace size) are
 * validated before anything is enqueued.  Per-tour contents (ids, costs,
 * lengths, demands) are validated on the device: a tour that fails gets
 * SPLIT_INF costs, SPLIT_SUM_INVALID as its sum and NaN as its mean.
 * The library reads the inputs and writes the outputs and workspace only
 * until the enqueued work completes.  Two calls sharing a workspace must
 * be ordered on one stream.
 */
int split_eval_device(const int32_t *d_tours, const int32_t *d_lens, int32_t num_tours,
                      int32_t max_len, const int32_t *d_dist, int32_t N,
                      const int16_t *d_demands, int64_t S, int32_t Q, int32_t *d_costs,
                      int64_t *d_sums, double *d_means, void *d_workspace, size_t ws_bytes,
                      split_stream_t stream);

/*
 * split_eval_path -- which kernels split_eval / split_eval_device run for a
 * call of this shape under the schedule in force (measurement and tests;
 * results never depend on it):
 *   SPLIT_PATH_ONE_LAUNCH  tables, recursion, exact fallback and the fold
 *                          in a single launch of one 8-wave workgroup, for
 *                          ONE tour with at most 256 recursion steps per
 *                          wave (ceil(ceil(S/64)/8) x max_len <= 256) and
 *                          N <= 256 (larger pools take the tour-ordered
 *                          path); automatic path choice only (a
 *                          path forced by split_set_schedule or a tuned
 *                          entry, or split_profile_enable, takes the general
 *                          kernels; the tuner records the one-launch form
 *                          as path 0 when it is the fastest)
 *   SPLIT_PATH_TILES       per-tour tables, one workgroup per 64-scenario
 *                          tile staged in LDS, exact fallback and fold
 *   SPLIT_PATH_ORDERED     as TILES, after the demands are rewritten in tour
 *                          order into the workspace
 * Returns the path (>= 0), or SPLIT_EINVAL for sizes split_eval_device
 * would reject.
 */
#define SPLIT_PATH_ONE_LAUNCH 0
#define SPLIT_PATH_TILES 1
#define SPLIT_PATH_ORDERED 2

int split_eval_path(int32_t num_tours, int32_t max_len, int32_t N, int64_t S, int32_t Q);

/*
 * Route recovery (App. A: the giant tour is cut into routes by the split
 * operator; App. B: a batched DP that records each minimiser and is then
 * backtracked recovers the decisions).  For ONE giant tour over every
 * scenario s:
 *   pred_s(i) = the smallest p with V_s(i) = V_s(p) + W(p,i), admissible
 *               (ties go to the longest last route), or SPLIT_NO_PRED when
 *               V_s(i) = +inf;
 *   cut points i_k = n, i_{k-1} = pred_s(i_k), ..., down to 0; route r
 *   covers tour positions i_{r-1}+1 .. i_r (i_0 = 0).
 *
 * split_routes_device -- DEVICE pointers, enqueued on `stream` (nothing is
 * allocated, no host synchronisation).
 *   d_tour    int32 [n]          customer ids 1..N (n in [0, 65535])
 *   d_dist, N, d_demands, S, Q   as in split_eval (d_demands 16-byte aligned)
 *   d_costs   out int32 [S]      V_s(n), SPLIT_INF if no split exists
 *   d_pred    out uint16 [n*S]   POSITION-MAJOR: d_pred[(i-1)*S + s] = pred_s(i)
 *   d_cuts    out uint16 [n*S]   POSITION-MAJOR: d_cuts[(r-1)*S + s] = i_r for
 *                                r = 1..nroutes_s (increasing); entries past
 *                                nroutes_s are not written
 *   d_nroutes out int32 [S]      number of routes k (0 when V_s(n) = +inf
 *                                or n = 0; -1 when the inputs failed
 *                                device-side validation)
 *   d_workspace, ws_bytes        caller-owned device scratch of at least
 *                                split_routes_workspace_bytes(n, N, S)
 *                                bytes, 256-byte aligned
 * d_tour, d_pred and d_cuts may be NULL when n = 0.  Host-checkable
 * arguments are validated before anything is enqueued (SPLIT_EINVAL).  The
 * tour's ids, costs and the int32 guard, and the demands' signs, are
 * checked on the device: on failure every d_costs entry is SPLIT_INF and
 * every d_nroutes entry -1.  The library touches the buffers only until
 * the enqueued work completes; two calls sharing a workspace must be
 * ordered on one stream.  Tiles whose 64 x N demand bytes do not fit in
 * LDS, whose demands exceed 255, or whose windows exceed the register
 * ring are recomputed by an exact (slower) kernel; results never depend
 * on the path taken.  Long tours on large pools (more than 16 KB of demand
 * bytes per 64-scenario tile) take a path that first writes the tour's
 * demands in tour order into the workspace, one byte per position, and
 * streams them from there (the workspace then includes S x (n rounded up
 * to 32, plus 32) bytes for that copy).
 */
#define SPLIT_NO_PRED 0xFFFF

size_t split_routes_workspace_bytes(int32_t n, int32_t N, int64_t S);
int split_routes_device(const int32_t *d_tour, int32_t n, const int32_t *d_dist, int32_t N,
                        const int16_t *d_demands, int64_t S, int32_t Q, int32_t *d_costs,
                        uint16_t *d_pred, uint16_t *d_cuts, int32_t *d_nroutes,
                        void *d_workspace, size_t ws_bytes, split_stream_t stream);

/*
 * split_routes_set_variant -- window variant of the route-recovery kernel
 * for every later call in the process, with the meaning of
 * split_set_schedule's first four arguments (ring 32 or 64, first head
 * group, later head groups, exit spacing).  ring = 0 restores the automatic
 * choice (by Q).  SPLIT_EINVAL for a variant that is not compiled in.
 * The recursion carries each potential and its predecessor in one int32
 * key when the tour's costs allow it (3 n maxcost < 2^23 for ring 32,
 * 2^22 for ring 64); other tours (up to the general 2^29 guard) take a
 * slower path of the same ring length that tracks the predecessor per
 * cell.  split_routes_list_variants writes up to `cap` entries of 4 int32
 * {ring, first, group, every} to `out` (host memory) and returns the number
 * compiled in.  Not thread-safe against concurrent calls.
 */
int split_routes_set_variant(int32_t ring, int32_t first, int32_t group, int32_t every);
int split_routes_list_variants(int32_t *out, int32_t cap);

/*
 * split_routes_set_path -- how later route-recovery calls in the process
 * read the demands: 0 automatic (by the demand bytes per tile), 1 the tile
 * staged in LDS, 2 the tour-ordered copy in the workspace (taken only where
 * its permute tile, 64 x N demand bytes, fits in LDS; else path 1).
 * split_routes_workspace_bytes reflects the setting: query it after
 * setting the path.  SPLIT_EINVAL outside [0, 2].  Results never depend on
 * the path.  Not thread-safe against concurrent calls.
 */
int split_routes_set_path(int32_t path);

/*
 * Full value table (Sec. 2.3 recursion; the batched DP of App. A returns
 * the value array over every tour position and scenario, of which the
 * evaluation entry points keep only V_s(n)).  For ONE giant tour over
 * every scenario s:
 *   V_s(j) = min over admissible p < j of V_s(p) + W(p,j), V_s(0) = 0,
 *   for j = 1..n, SPLIT_INF where no split of the first j customers exists.
 *
 * split_values_device -- DEVICE pointers, enqueued on `stream` (nothing is
 * allocated):
 *   d_tour, n, d_dist, N, d_demands, S, Q   as in split_routes_device
 *   d_V       out int32 [n*S]  POSITION-MAJOR: d_V[(j-1)*S + s] = V_s(j)
 *   d_status  out int32 [1]    0, or 1 when a negative demand was read (the
 *                              entries of such a scenario are SPLIT_INF)
 *   d_workspace, ws_bytes      caller-owned device scratch of at least
 *                              split_values_workspace_bytes(n, N, S) bytes,
 *                              256-byte aligned
 * d_tour and d_V may be NULL when n = 0.  Host-checkable arguments are
 * validated before anything is enqueued (SPLIT_EINVAL).  The tour's ids,
 * costs and the int32 guard are checked on the device: on failure every
 * entry is SPLIT_INF.  The recursion runs exactly from its definition (one
 * read of V_s(p) and of one demand per admissible predecessor), reading
 * back the rows it has written: an inspection output, slower than the
 * evaluation kernels, which never materialise the table.  The library
 * touches the buffers only until the enqueued work completes; two calls
 * sharing a workspace must be ordered on one stream.
 */
size_t split_values_workspace_bytes(int32_t n, int32_t N, int64_t S);
int split_values_device(const int32_t *d_tour, int32_t n, const int32_t *d_dist, int32_t N,
                        const int16_t *d_demands, int64_t S, int32_t Q, int32_t *d_V,
                        int32_t *d_status, void *d_workspace, size_t ws_bytes,
                        split_stream_t stream);

/*
 * Split variants (App. A, the extensive form: its objective charges every
 * vehicle's overload l_k at rate beta, and its fleet-size constraint allows
 * at most K vehicles).  For ONE giant tour over every scenario s, with
 *   cost(p,i) = W(p,i) + beta * max(0, load_s(p+1..i) - Q)   (beta >= 0),
 *   cost(p,i) = W(p,i) if load_s(p+1..i) <= Q, else excluded (beta < 0),
 * and J_k(i) the cheapest split of positions 1..i into exactly k routes
 * (J_0(0) = 0, J_k(i) = min_{p<i} J_{k-1}(p) + cost(p,i)), the scenario's
 * cost is min_{k<=K} J_k(n); K = 0 means an unlimited fleet.  beta < 0 with
 * K = 0 is the plain split of split_eval.
 *
 * split_variant_device -- DEVICE pointers, enqueued on `stream`, nothing
 * allocated.
 *   d_tour    int32 [n]      customer ids 1..N (may be NULL when n = 0)
 *   d_dist, N, d_demands, S, Q  as in split_eval (d_demands 16-byte aligned)
 *   beta      penalty per unit of overload, in [0, 2^24); negative = hard
 *   K         fleet bound in [0, 65535]; 0 = unlimited
 *   d_costs   out int32 [S]  the scenario's cost, SPLIT_INF if no split
 *                            exists (hard capacity, or fewer than needed
 *                            vehicles)
 *   d_status  out int32 [1]  0, or a bit set: 1 invalid tour or costs past
 *                            the int32 guard, 2 negative demand, 4 a
 *                            scenario's penalty range past the int32 guard
 *                            (3 n maxcost + beta (load + Q) >= 2^29 or
 *                            load + Q >= 2^24); when non-zero every cost is
 *                            SPLIT_INF
 *   d_workspace, ws_bytes    caller-owned device scratch of at least
 *                            split_variant_workspace_bytes(n, N, S, K) bytes,
 *                            256-byte aligned (K > 0 adds 8 n S bytes for
 *                            the potentials of consecutive passes)
 * Host-checkable arguments are validated before anything is enqueued
 * (SPLIT_EINVAL).  The library touches the buffers only until the enqueued
 * work completes; two calls sharing a workspace must be ordered on one
 * stream.  Windows longer than the register ring and demands above 255
 * take an exact (slower) kernel.  The demands are read from a tile staged
 * in LDS, or, for long tours on large pools and tours over at most half of
 * the pool, from a tour-ordered copy (one byte per position) written into
 * the workspace, which then includes S x (n rounded up to 32, plus 32)
 * bytes for it; results never depend on the path.
 */
size_t split_variant_workspace_bytes(int32_t n, int32_t N, int64_t S, int32_t K);
int split_variant_device(const int32_t *d_tour, int32_t n, const int32_t *d_dist, int32_t N,
                         const int16_t *d_demands, int64_t S, int32_t Q, int32_t beta, int32_t K,
                         int32_t *d_costs, int32_t *d_status, void *d_workspace, size_t ws_bytes,
                         split_stream_t stream);

/*
 * split_variant_set_path -- how later split-variant calls in the process
 * read the demands, with split_routes_set_path's meaning (0 automatic,
 * 1 the tile in LDS, 2 the tour-ordered copy where its permute tile fits).
 * split_variant_workspace_bytes reflects the setting.  SPLIT_EINVAL outside
 * [0, 2].  Not thread-safe against concurrent calls.
 */
int split_variant_set_path(int32_t path);

/*
 * Min-plus Bellman updates (Sec. 2, min-plus matrix formulation: the
 * stage-wise update J_{t+1} = A_t^T (x) J_t in the (min, +) semiring; App. A
 * gives a worked 3-to-2-state example and the scenario-batched forward DP).
 * For each of B independent problems (scenarios, or customer-scenario
 * pairs) with m states per stage:
 *   J_{t+1}(j) = min_i A_t(i, j) + J_t(i),   t = 0..T-1.
 * Values are non-negative int32; INT32_MAX is +inf (a negative entry reads
 * as +inf), and a finite sum that reaches INT32_MAX is +inf.
 *
 * split_minplus_forward_device -- DEVICE pointers, enqueued on `stream`.
 *   d_A     int32, row-major (source i, target j): [T][m][m] when shared = 1
 *           (one matrix per stage for every problem), [T][B][m][m] when
 *           shared = 0
 *   d_J0    int32 [B][m]  initial cost-to-go (INT32_MAX where not allowed)
 *   d_JT    out int32 [B][m]  J_T
 *   d_arg   out int32 [T][B][m] (may be NULL): the smallest i attaining
 *           J_{t+1}(j), -1 where J_{t+1}(j) is +inf
 *   1 <= m <= 4096, T >= 1, 1 <= B < 2^31.  Returns SPLIT_EINVAL on bad
 *   sizes or null required pointers, before anything is enqueued.
 *
 * split_minplus_backtrack_device -- the optimal state path of every problem
 * (App. B: backtracking the recorded minimisers):
 *   d_path  out int32 [T+1][B]: d_path[T][b] = the smallest j minimising
 *           J_T(b, j); d_path[t][b] = d_arg[t][b][d_path[t+1][b]]; -1
 *           throughout when J_T(b, .) is +inf everywhere.
 *
 * split_ou_transitions_device -- the transition matrices of the
 * order-up-to inventory instance (App. B: a customer is replenished up to
 * its capacity U or not at all; the illustrative matrix form), written as
 * d_A [T][B][U+1][U+1] for split_minplus_forward_device (shared = 0).
 * States are end-of-day inventories 0..U.  From inventory I with day
 * demand d the delivery is q = 0 or q = U - I, the next state
 * max(0, I + q - d), and the day costs
 *   transport(q) + h[next] + rho * max(0, d - I - q),
 * transport(0) = 0, transport(q > 0) = (the cheapest of the day's R route
 * options whose residual capacity is at least q) + u * q, impossible when
 * none has room.  A(I, J) is the cheapest choice landing in J, INT32_MAX if
 * none (sums are formed in 64 bits and saturate at INT32_MAX).
 *   d_demand   int32 [T][B]        demands, >= 0
 *   d_opt_cost int32 [T][B][R]     insertion cost of each route option, >= 0
 *   d_opt_cap  int32 [T][B][R]     residual capacity of each route option
 *   d_h        int32 [U+1]         end-of-day cost of each inventory level
 *   u, rho     unit transport cost and unit shortage penalty, >= 0
 *   0 <= U < 4096, 1 <= R <= 64.
 */
int split_minplus_forward_device(const int32_t *d_A, int32_t shared, int32_t T, int32_t m,
                                 int64_t B, const int32_t *d_J0, int32_t *d_JT, int32_t *d_arg,
                                 split_stream_t stream);
int split_minplus_backtrack_device(const int32_t *d_JT, const int32_t *d_arg, int32_t T,
                                   int32_t m, int64_t B, int32_t *d_path, split_stream_t stream);
int split_ou_transitions_device(int32_t U, int32_t T, int64_t B, int32_t R,
                                const int32_t *d_demand, const int32_t *d_opt_cost,
                                const int32_t *d_opt_cap, const int32_t *d_h, int32_t u,
                                int32_t rho, int32_t *d_A, split_stream_t stream);

/*
 * split_ou_dp_device -- the whole order-up-to inventory DP in one launch
 * (App. B: the illustrative matrix form and its note on parallelism over
 * scenarios x transitions x route options, with the minimum taken first
 * over route options and then over predecessor states; the batched DP
 * records its minimisers).  For valid inputs the results are exactly those
 * of split_ou_transitions_device followed by split_minplus_forward_device
 * (shared = 0) on the same arguments, but no transition matrix is formed:
 * from level I with day demand d the no-delivery action lands on
 * max(0, I - d) and the delivery of U - I on max(0, U - d), so each level
 * has one no-delivery predecessor (level 0: every I <= d) and the delivery
 * level every I < U.
 *   d_demand, d_opt_cost, d_opt_cap, d_h, u, rho: as split_ou_transitions_device
 *   d_J0     int32 [B][U+1]  initial cost-to-go (INT32_MAX where not allowed;
 *            a negative entry reads as +inf)
 *   d_JT     out int32 [B][U+1]  J_T
 *   d_arg    out int32 [T][B][U+1] (may be NULL): the smallest predecessor
 *            level attaining J_{t+1}(J), -1 where it is +inf (the layout of
 *            split_minplus_forward_device, so split_minplus_backtrack_device
 *            recovers the state paths)
 *   d_status out int32 (may be NULL): 0, or 1 when a negative demand,
 *            option cost or h entry was read (results then unspecified;
 *            every access stays in bounds)
 *   0 <= U <= 31, T >= 1, 1 <= B < 2^31, 1 <= R <= 64, u, rho >= 0.
 * Device pointers, enqueued on `stream`; SPLIT_EINVAL on bad sizes or null
 * required pointers, before anything is enqueued.
 */
int split_ou_dp_device(int32_t U, int32_t T, int64_t B, int32_t R, const int32_t *d_demand,
                       const int32_t *d_opt_cost, const int32_t *d_opt_cap, const int32_t *d_h,
                       int32_t u, int32_t rho, const int32_t *d_J0, int32_t *d_JT,
                       int32_t *d_arg, int32_t *d_status, split_stream_t stream);

/*
 * First-stage candidate search: a genetic algorithm over giant tours whose
 * candidates are all evaluated on every scenario by the batched split (the
 * paper's candidate-based scheme, Sec. 4 "decision quality under fixed
 * time budgets"; the appendix tables of candidates explored vs objective).
 * (mu + lambda) generations: binary-tournament parents on the exact
 * scenario sum, order crossover, a random segment reversal with probability
 * `mutation`, the `offspring` children of a generation evaluated in one
 * batched call, and the best `population` of parents and children kept
 * (stable: on equal sums parents first).  Deterministic for a seed
 * (splitmix64 stream); with the same seed two evaluators that return the
 * same sums give the same search.
 */
typedef struct {
    int32_t population;   /* tours kept per generation (mu), >= 2 */
    int32_t offspring;    /* candidates evaluated per generation (lambda), >= 1 */
    int32_t generations;  /* generation limit; <= 0: none */
    double time_budget_s; /* wall-clock limit in seconds; <= 0: none (one limit is required) */
    double mutation;      /* probability of a segment reversal per child, in [0, 1] */
    uint64_t seed;        /* random stream */
} split_search_params;

/* Caller-supplied evaluator: exact scenario sums of `count` host tours of n
 * customers each (tours[k*n .. k*n+n-1]); INT64_MAX for an infeasible tour;
 * returns 0 on success. */
typedef int (*split_search_eval_fn)(void *ctx, const int32_t *tours, int32_t count, int32_t n,
                                    int64_t *sums);

/*
 * split_search_run -- runs the search over permutations of customers 1..N.
 *   d_dist, d_demands, S, Q  DEVICE inputs as in split_eval_device (used by
 *            the built-in evaluator: one captured evaluation plan per batch
 *            size, on `stream`, buffers allocated and freed by the call)
 *   init_tour   host int32 [N], a permutation seeding the population (may be NULL)
 *   evaluator, evaluator_ctx  optional host evaluator replacing the GPU one
 *   best_tour   out host int32 [N]; best_sum  out: its scenario sum
 *   candidates  out: tours evaluated (population + generations * offspring)
 *   trace       out host double [trace_cap][3] (may be NULL if trace_cap = 0):
 *               per generation (0 = initial population) the elapsed seconds,
 *               the candidates evaluated so far and the best sum
 *   trace_len   out: generations recorded (may exceed trace_cap)
 * SPLIT_EINVAL for bad parameters or an init_tour that is not a permutation;
 * errors of the evaluator are returned as they come.  Synchronous.
 */
int split_search_run(const int32_t *d_dist, int32_t N, const int16_t *d_demands, int64_t S,
                     int32_t Q, const int32_t *init_tour, const split_search_params *params,
                     split_search_eval_fn evaluator, void *evaluator_ctx, int32_t *best_tour,
                     int64_t *best_sum, int64_t *candidates, double *trace, int32_t trace_cap,
                     int32_t *trace_len, split_stream_t stream);

/*
 * split_count_cells_device -- Bellman-cell counter (measurement utility).
 * For each tour writes the number of capacity-admissible relaxations
 * (s, p, i), i.e. sum over scenarios and positions i of the number of
 * predecessors p < i whose route p+1..i has load <= Q.  Device pointers,
 * enqueued on `stream`; d_cells is int64 [num_tours].  Tours must already
 * be valid (no device-side validation).
 */
int split_count_cells_device(const int32_t *d_tours, const int32_t *d_lens, int32_t num_tours,
                             int32_t N, const int16_t *d_demands, int64_t S, int32_t Q,
                             int64_t *d_cells, split_stream_t stream);

/*
 * split_set_schedule -- schedule override for every later call in the
 * process (the tuner uses it).  ring = 32 or 64 is the register-ring length
 * of the main kernel (longer windows are recomputed by the exact fallback,
 * so results never depend on it); first = cells of the first head group,
 * validated with one check issued a position early; group = cells of each
 * later head group, validated with one check each (0 = none); every = tail
 * cells between exits on an empty lane mask; waves = tours per workgroup
 * that share one staged scenario tile (1, 2, 4 or 8; 0 = automatic); path =
 * 1 stages whole scenario rows in LDS and gathers through the tour, 2 first
 * rewrites the demands in tour order and streams them (0 = automatic, by
 * the LDS each wave would need).  ring = 0 restores the automatic choice.
 * split_workspace_bytes accounts for the override in force when called.
 * A (ring, first, group, every) window variant that is not compiled in
 * returns SPLIT_EINVAL.  Not thread-safe against concurrent evaluations.
 */
int split_set_schedule(int32_t ring, int32_t first, int32_t group, int32_t every, int32_t waves,
                       int32_t path);

/*
 * split_list_variants -- the compiled window variants, for split_set_schedule.
 * Writes up to `cap` entries of 4 int32 {ring, first, group, every} to
 * `out` (host memory, caller-owned, 4*cap words; may be NULL when cap = 0)
 * and returns the total number compiled in (which may exceed cap).
 */
int split_list_variants(int32_t *out, int32_t cap);

/*
 * Autotuning.  split_tune_device times every compiled schedule (ring length,
 * head/tail structure, tours per workgroup, fused or ordered path, and the
 * one-launch form where the shape allows it, recorded as path 0) on the
 * given device inputs, `reps` timed launches each after two warm-ups, on
 * `stream` (synchronising it), and records the fastest for the call's shape
 * bucket (tour count, length, pool size, scenario count and capacity, each
 * bucketed logarithmically); later calls in the bucket use it unless
 * split_set_schedule overrides.  Every candidate is parity-gated: its costs
 * and sums must equal the automatic schedule's bit for bit, else
 * SPLIT_EDEVICE is returned and nothing is recorded.  It allocates its own
 * device buffers.  best_ms (may be NULL) receives the winner's time per
 * evaluation.  split_tune_lookup reports the recorded schedule as
 * {ring, first, group, every, waves, path} (SPLIT_EAGAIN if none);
 * split_tune_save / split_tune_load write / read the table as text;
 * split_tune_clear forgets it.
 */
int split_tune_device(const int32_t *d_tours, const int32_t *d_lens, int32_t num_tours,
                      int32_t max_len, const int32_t *d_dist, int32_t N,
                      const int16_t *d_demands, int64_t S, int32_t Q, int32_t reps,
                      split_stream_t stream, double *best_ms);
int split_tune_lookup(int32_t num_tours, int32_t max_len, int32_t N, int64_t S, int32_t Q,
                      int32_t sched[6]);
int split_tune_save(const char *path);
int split_tune_load(const char *path);
int split_tune_clear(void);

/*
 * split_probe_valu_peak -- measured int32 vector-ALU rate of the current
 * device, as a roofline reference (a measurement helper, not part of the
 * method).  Runs a kernel of independent v_min_i32 chains with eight waves
 * per SIMD on `stream`, waits for it, and stores lane-operations per second
 * in *lane_ops_per_s (host pointer).  Allocates and frees a 4-byte device
 * buffer.  SPLIT_EINVAL for a null pointer, SPLIT_EDEVICE/ENOMEM on device
 * errors.
 */
int split_probe_valu_peak(double *lane_ops_per_s, split_stream_t stream);

/*
 * Measurement.  While enabled, every launch of the main evaluation kernel
 * is bracketed by a pair of HIP events recorded on the launch stream.
 * split_profile_read waits for the recorded events, returns the summed
 * elapsed milliseconds and the number of launches since the previous read,
 * and resets both.  Disabled by default; do not enable it for calls that
 * are being captured into a graph.
 */
int split_profile_enable(int32_t on);
int split_profile_read(double *kernel_ms, int64_t *launches);

/*
 * Plans: the batched form.  A plan binds one set of device buffers and
 * sizes, owns its workspace, and captures the evaluation into a HIP graph
 * once; split_plan_launch replays it.  Rewriting the contents of d_tours,
 * d_lens (within max_len), d_demands between launches is allowed (the GA
 * pattern: new candidate tours, same shapes).  split_plan_launch_eager
 * enqueues the same evaluation (same buffers, schedule and workspace) as
 * ordinary kernel launches on `stream` instead of a graph launch: the same
 * results, with the host-side cost of one library call and no graph
 * launch, which is the lower latency for evaluations of a few kernels'
 * length.  Launches of one plan on different streams must not overlap
 * (they share the workspace and outputs).
 */
int split_plan_create(split_plan **plan, const int32_t *d_tours, const int32_t *d_lens,
                      int32_t num_tours, int32_t max_len, const int32_t *d_dist, int32_t N,
                      const int16_t *d_demands, int64_t S, int32_t Q, int32_t *d_costs,
                      int64_t *d_sums, double *d_means, split_stream_t stream);
int split_plan_launch(split_plan *plan, split_stream_t stream);
int split_plan_launch_eager(split_plan *plan, split_stream_t stream);
int split_plan_destroy(split_plan *plan);

/*
 * split_eval_device_noalloc -- split_eval_device for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid allocation): the same arguments less the
 * workspace, whose role a fixed device array inside the library takes
 * (SPLIT_NOALLOC_SCRATCH_BYTES, 32 MiB; each device the library runs on
 * holds its own copy until the process ends).  The call allocates nothing
 * and issues no memset: the kernels clear what must start at zero.  Calls
 * whose workspace (as split_workspace_bytes sizes it for the tile path)
 * exceeds the array return SPLIT_EINVAL naming both sizes, before anything
 * is enqueued; the tour-ordered demand copy is never used, so every call
 * stages tiles in LDS.  Results equal split_eval_device's.  Calls that
 * overlap on one device share the array and race: serialise them (one
 * stream, or events) per device.
 * split_noalloc_scratch_bytes returns the array's size.
 */
#define SPLIT_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int split_eval_device_noalloc(const int32_t *d_tours, const int32_t *d_lens, int32_t num_tours,
                              int32_t max_len, const int32_t *d_dist, int32_t N,
                              const int16_t *d_demands, int64_t S, int32_t Q, int32_t *d_costs,
                              int64_t *d_sums, double *d_means, split_stream_t stream);
size_t split_noalloc_scratch_bytes(void);

/*
 * Served form (the serving loop around the split operator; the paper's
 * batch loop in App. B sizes batches from free GPU memory and retries
 * smaller batches on out-of-memory): continuous batching of evaluation
 * requests under an HBM budget, drained at the granularity of a tile of 64
 * scenarios.
 *
 * split_server_create reserves the server's device memory: `budget_bytes`
 *   (0 = three quarters of the free device memory), retried at half the
 *   size while the reservation fails with out-of-memory (down to 64 MiB);
 *   split_server_stats reports what was reserved.  `max_len` is the longest
 *   tour the server accepts (1..65535; it sizes the exact-fallback scratch).
 * split_server_add_instance registers an instance: `dist` (host, int32
 *   [(N+1)*(N+1)]) is copied and kept on the host, where each request's
 *   tour constants are computed; `demands` (host, int16 [S*N]
 *   scenario-major) are copied into the budget and stay resident until
 *   split_server_remove_instance (which takes effect once no request uses
 *   them).  SPLIT_ENOMEM if they can never fit, SPLIT_EAGAIN if the budget
 *   has no room for them now.
 * split_server_submit queues one giant tour (host pointer, ids in [1, N],
 *   copied; validated as split_eval's host form) for evaluation on a
 *   resident instance with capacity Q, and returns a request id at once.
 *   costs_out is an optional HOST buffer of S int32, filled before
 *   completion is reported.
 * split_server_submit_copy is the same for a request that brings its own
 *   instance (host pointers, copied at submission): its demands are copied
 *   to the device at admission and counted until it completes.
 *   A request is admitted in arrival order once its footprint (tables,
 *   outputs, the tour-ordered demand copy for pools above 256 customers,
 *   its own demands if any) fits; admitted requests' tiles join the device
 *   work queue while earlier requests are still running.
 * split_server_poll returns SPLIT_EAGAIN while the request is pending or
 *   running; once done it returns its sum and mean (as split_eval), its
 *   latency from submission to the result in seconds, and forgets the
 *   request.  A negative demand found on the device gives SPLIT_EINVAL.
 * split_server_wait blocks until the request is done (poll still needed).
 * split_server_destroy completes every admitted and pending request first.
 * Requests may be submitted and polled from several threads.
 */
typedef struct {
    int64_t submitted, completed, pending, running;
    size_t bytes_in_use, peak_bytes, capacity; /* arena bytes (the budget less fixed structures) */
    int64_t drains;                            /* drain launches so far */
    int64_t instances;                         /* resident instances */
    size_t deferred_bytes;  /* retired memory held until the drains running at retirement end */
    int64_t blocked_rounds; /* scheduler rounds in which the next request did not fit */
} split_server_stats_t;

int split_server_create(split_server **server, size_t budget_bytes, int32_t max_len);
int split_server_add_instance(split_server *server, const int32_t *dist, int32_t N,
                              const int16_t *demands, int64_t S, int64_t *instance_id);
int split_server_remove_instance(split_server *server, int64_t instance_id);
int split_server_submit(split_server *server, int64_t instance_id, const int32_t *tour,
                        int32_t n, int32_t Q, int32_t *costs_out, int64_t *request_id);
int split_server_submit_copy(split_server *server, const int32_t *tour, int32_t n,
                             const int32_t *dist, int32_t N, const int16_t *demands, int64_t S,
                             int32_t Q, int32_t *costs_out, int64_t *request_id);
int split_server_poll(split_server *server, int64_t request_id, int64_t *sum, double *mean,
                      double *latency_s);
int split_server_wait(split_server *server, int64_t request_id);
int split_server_stats(split_server *server, split_server_stats_t *stats);
int split_server_destroy(split_server *server);

/*
 * Test hook (for callers exercising the out-of-memory path): the library's
 * next `count` device reservations made by split_server_create report
 * out-of-memory, as a full device would.  0 turns it off.
 */
int split_debug_fail_allocations(int32_t count);

#ifdef __cplusplus
}
#endif

#endif /* SPLIT_EVAL_H */
