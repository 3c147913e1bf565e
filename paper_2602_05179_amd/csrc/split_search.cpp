// split_search.cpp -- first-stage candidate search: a genetic algorithm over
// giant tours whose candidates are evaluated by the scenario-batched split
// (the paper's candidate-based scheme: candidate first-stage decisions come
// from a genetic algorithm and every candidate is evaluated on all scenarios
// by the GPU; Sec. 4, decision quality under fixed time budgets, and the
// candidate-count tables of the appendix).
//
// Generation loop ((mu + lambda), deterministic for a seed):
//   * parents by binary tournament on the exact int64 scenario sum (lower is
//     better; equal sums keep the lower population index);
//   * order crossover: the child copies a random slice of parent 1 and
//     fills the other positions with parent 2's customers in parent 2's
//     order, starting after the slice;
//   * mutation with probability `mutation`: reversal of a random segment
//     (a 2-opt move on the giant tour);
//   * all offspring of a generation are evaluated in one batched call (one
//     replay of a captured evaluation plan on the GPU, or the caller's
//     evaluator), then the population keeps the best `population` of
//     parents and offspring (stable: parents first on equal sums).
// Random numbers: splitmix64 (Steele, Lea and Flood, 2014), one stream per
// run seeded by the caller.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <numeric>
#include <vector>

#include "split_eval.h"
#include "split_internal.h"

namespace {

struct SplitMix64 {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    // uniform integer in [0, n) (n >= 1), by rejection of the biased tail
    uint32_t below(uint32_t n)
    {
        const uint64_t lim = UINT64_MAX - UINT64_MAX % n;
        uint64_t x;
        do
            x = next();
        while (x >= lim);
        return (uint32_t)(x % n);
    }
    double unit() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

// Evaluates `count` tours of n customers each into exact scenario sums.
struct Evaluator {
    virtual ~Evaluator() = default;
    virtual int run(const int32_t *tours, int32_t count, int64_t *sums) = 0;
};

// GPU: one captured plan per batch size, tours copied in, sums copied out.
struct GpuEvaluator : Evaluator {
    const int32_t *d_dist;
    int32_t N;
    const int16_t *d_demands;
    int64_t S;
    int32_t Q;
    int32_t n;
    hipStream_t stream = nullptr;
    struct Slot {
        int32_t count = 0;
        int32_t *d_tours = nullptr, *d_lens = nullptr, *d_costs = nullptr;
        int64_t *d_sums = nullptr;
        double *d_means = nullptr;
        split_plan *plan = nullptr;
    };
    std::vector<Slot> slots;

    ~GpuEvaluator() override
    {
        for (Slot &s : slots) {
            if (s.plan)
                split_plan_destroy(s.plan);
            (void)hipFree(s.d_tours);
            (void)hipFree(s.d_lens);
            (void)hipFree(s.d_costs);
            (void)hipFree(s.d_sums);
            (void)hipFree(s.d_means);
        }
    }

    int slot_for(int32_t count, Slot **out)
    {
        for (Slot &s : slots)
            if (s.count == count) {
                *out = &s;
                return SPLIT_OK;
            }
        Slot s;
        s.count = count;
        const size_t ts = (size_t)count * n * sizeof(int32_t);
        if (hipMalloc(&s.d_tours, ts ? ts : 4) != hipSuccess ||
            hipMalloc(&s.d_lens, (size_t)count * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&s.d_costs, (size_t)count * S * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&s.d_sums, (size_t)count * sizeof(int64_t)) != hipSuccess ||
            hipMalloc(&s.d_means, (size_t)count * sizeof(double)) != hipSuccess) {
            slots.push_back(s); // freed by the destructor
            return splitk::set_error(SPLIT_ENOMEM, "search: device buffers");
        }
        std::vector<int32_t> lens(count, n);
        if (hipMemcpy(s.d_lens, lens.data(), (size_t)count * sizeof(int32_t),
                      hipMemcpyHostToDevice) != hipSuccess) {
            slots.push_back(s);
            return splitk::set_error(SPLIT_EDEVICE, "search: copy lengths");
        }
        const int rc = split_plan_create(&s.plan, s.d_tours, s.d_lens, count, n, d_dist, N,
                                         d_demands, S, Q, s.d_costs, s.d_sums, s.d_means, stream);
        slots.push_back(s);
        if (rc != SPLIT_OK)
            return rc;
        *out = &slots.back();
        return SPLIT_OK;
    }

    int run(const int32_t *tours, int32_t count, int64_t *sums) override
    {
        Slot *s = nullptr;
        int rc = slot_for(count, &s);
        if (rc != SPLIT_OK)
            return rc;
        if (hipMemcpyAsync(s->d_tours, tours, (size_t)count * n * sizeof(int32_t),
                           hipMemcpyHostToDevice, stream) != hipSuccess)
            return splitk::set_error(SPLIT_EDEVICE, "search: copy tours");
        rc = split_plan_launch(s->plan, stream);
        if (rc != SPLIT_OK)
            return rc;
        if (hipMemcpyAsync(sums, s->d_sums, (size_t)count * sizeof(int64_t),
                           hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return splitk::set_error(SPLIT_EDEVICE, "search: copy sums");
        for (int32_t k = 0; k < count; ++k)
            if (sums[k] == SPLIT_SUM_INVALID)
                return splitk::set_error(SPLIT_EINVAL, "search: invalid input on the device");
        return SPLIT_OK;
    }
};

struct CallbackEvaluator : Evaluator {
    split_search_eval_fn fn;
    void *ctx;
    int32_t n;
    int run(const int32_t *tours, int32_t count, int64_t *sums) override
    {
        const int rc = fn(ctx, tours, count, n, sums);
        return rc == 0 ? SPLIT_OK : splitk::set_error(SPLIT_EDEVICE, "search: evaluator returned %d", rc);
    }
};

void order_crossover(const int32_t *p1, const int32_t *p2, int32_t n, SplitMix64 &rng,
                     std::vector<uint8_t> &used, int32_t *child, int32_t N)
{
    uint32_t a = rng.below((uint32_t)n), b = rng.below((uint32_t)n);
    if (a > b)
        std::swap(a, b);
    std::fill(used.begin(), used.end(), 0);
    for (uint32_t k = a; k <= b; ++k) {
        child[k] = p1[k];
        used[p1[k]] = 1;
    }
    int32_t pos = (int32_t)((b + 1) % n);
    for (int32_t k = 0; k < n; ++k) {
        const int32_t c = p2[(b + 1 + k) % n];
        if (used[c])
            continue;
        child[pos] = c;
        used[c] = 1;
        pos = (pos + 1) % n;
    }
    (void)N;
}

int run_search(Evaluator &ev, int32_t N, const int32_t *init_tour, const split_search_params &p,
               int32_t *best_tour, int64_t *best_sum, int64_t *candidates, double *trace,
               int32_t trace_cap, int32_t *trace_len)
{
    const int32_t n = N, P = p.population, C = p.offspring;
    SplitMix64 rng{p.seed};
    std::vector<int32_t> pop((size_t)P * n), kids((size_t)C * n);
    std::vector<int64_t> pop_sum(P), kid_sum(C);
    for (int32_t i = 0; i < P; ++i) {
        int32_t *t = &pop[(size_t)i * n];
        if (i == 0 && init_tour) {
            std::copy(init_tour, init_tour + n, t);
            continue;
        }
        std::iota(t, t + n, 1);
        for (int32_t k = n - 1; k > 0; --k) // Fisher-Yates
            std::swap(t[k], t[rng.below((uint32_t)k + 1)]);
    }
    const auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&]() {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    };
    int rc = ev.run(pop.data(), P, pop_sum.data());
    if (rc != SPLIT_OK)
        return rc;
    int64_t evaluated = P;
    int32_t tl = 0;
    auto best_index = [&]() {
        return (int32_t)(std::min_element(pop_sum.begin(), pop_sum.end()) - pop_sum.begin());
    };
    auto record = [&]() {
        if (trace && tl < trace_cap) {
            trace[3 * tl] = elapsed();
            trace[3 * tl + 1] = (double)evaluated;
            trace[3 * tl + 2] = (double)pop_sum[best_index()];
        }
        ++tl;
    };
    record();
    std::vector<uint8_t> used((size_t)N + 1);
    std::vector<int32_t> order((size_t)P + C);
    std::vector<int32_t> next((size_t)P * n);
    std::vector<int64_t> next_sum(P);
    for (int32_t g = 0; p.generations <= 0 || g < p.generations; ++g) {
        if (p.time_budget_s > 0 && elapsed() >= p.time_budget_s)
            break;
        auto tournament = [&]() {
            const int32_t x = (int32_t)rng.below((uint32_t)P), y = (int32_t)rng.below((uint32_t)P);
            return (pop_sum[y] < pop_sum[x] || (pop_sum[y] == pop_sum[x] && y < x)) ? y : x;
        };
        for (int32_t c = 0; c < C; ++c) {
            const int32_t a = tournament(), b = tournament();
            int32_t *child = &kids[(size_t)c * n];
            order_crossover(&pop[(size_t)a * n], &pop[(size_t)b * n], n, rng, used, child, N);
            if (rng.unit() < p.mutation) {
                uint32_t i = rng.below((uint32_t)n), j = rng.below((uint32_t)n);
                if (i > j)
                    std::swap(i, j);
                std::reverse(child + i, child + j + 1);
            }
        }
        rc = ev.run(kids.data(), C, kid_sum.data());
        if (rc != SPLIT_OK)
            return rc;
        evaluated += C;
        // (mu + lambda): stable order on the sum, parents before offspring
        std::iota(order.begin(), order.end(), 0);
        auto sum_of = [&](int32_t k) { return k < P ? pop_sum[k] : kid_sum[k - P]; };
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t x, int32_t y) { return sum_of(x) < sum_of(y); });
        for (int32_t i = 0; i < P; ++i) {
            const int32_t k = order[i];
            const int32_t *src = k < P ? &pop[(size_t)k * n] : &kids[(size_t)(k - P) * n];
            std::copy(src, src + n, &next[(size_t)i * n]);
            next_sum[i] = sum_of(k);
        }
        pop.swap(next);
        pop_sum.swap(next_sum);
        record();
    }
    const int32_t bi = best_index();
    std::copy(&pop[(size_t)bi * n], &pop[(size_t)bi * n] + n, best_tour);
    *best_sum = pop_sum[bi];
    *candidates = evaluated;
    *trace_len = tl;
    return SPLIT_OK;
}

} // namespace

extern "C" {

int split_search_run(const int32_t *d_dist, int32_t N, const int16_t *d_demands, int64_t S,
                     int32_t Q, const int32_t *init_tour, const split_search_params *params,
                     split_search_eval_fn evaluator, void *evaluator_ctx, int32_t *best_tour,
                     int64_t *best_sum, int64_t *candidates, double *trace, int32_t trace_cap,
                     int32_t *trace_len, split_stream_t stream)
{
    splitk::clear_error();
    if (!params || !best_tour || !best_sum || !candidates || !trace_len)
        return splitk::set_error(SPLIT_EINVAL, "null pointer argument");
    const split_search_params &p = *params;
    if (N < 2 || S < 1 || Q < 0 || p.population < 2 || p.offspring < 1 ||
        p.mutation < 0.0 || p.mutation > 1.0 || (p.generations <= 0 && p.time_budget_s <= 0) ||
        trace_cap < 0 || (trace_cap > 0 && !trace) || N > splitk::kMaxLen)
        return splitk::set_error(SPLIT_EINVAL,
                                 "need N >= 2, S >= 1, Q >= 0, population >= 2, offspring >= 1, "
                                 "mutation in [0,1], a generation or time limit");
    if (init_tour) {
        std::vector<uint8_t> seen((size_t)N + 1, 0);
        for (int32_t k = 0; k < N; ++k) {
            const int32_t c = init_tour[k];
            if (c < 1 || c > N || seen[c])
                return splitk::set_error(SPLIT_EINVAL, "init_tour must be a permutation of 1..N");
            seen[c] = 1;
        }
    }
    if (evaluator) {
        CallbackEvaluator ev;
        ev.fn = evaluator;
        ev.ctx = evaluator_ctx;
        ev.n = N;
        return run_search(ev, N, init_tour, p, best_tour, best_sum, candidates, trace, trace_cap,
                          trace_len);
    }
    if (!d_dist || !d_demands)
        return splitk::set_error(SPLIT_EINVAL, "null device pointer argument");
    GpuEvaluator ev;
    ev.d_dist = d_dist;
    ev.N = N;
    ev.d_demands = d_demands;
    ev.S = S;
    ev.Q = Q;
    ev.n = N;
    ev.stream = static_cast<hipStream_t>(stream);
    return run_search(ev, N, init_tour, p, best_tour, best_sum, candidates, trace, trace_cap,
                      trace_len);
}

} // extern "C"
