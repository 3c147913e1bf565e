// split_routes.hip -- route recovery: the per-scenario minimising
// predecessors of the split recursion and the route cut points obtained by
// backtracking them (the giant tour is cut into routes by the split, App. A;
// a batched DP that records its minimisers is backtracked to recover the
// decisions, App. B).
//
// Recursion and potential form as in split_kernels.hip: with
// f_p = V(p) + a_{p+1}, position i takes m_i = min over the admissible
// window of f_p, and pred(i) is the SMALLEST admissible p with f_p = m_i
// (among equal route costs the longest last route).  Equal f_p means equal
// V(p) + W(p,i), since b_i is common to the window, so the tie-break is
// exact.
//
// Packed keys (the main path).  Each ring slot holds
//   K_p = f_p * 2^B + (p - base),   B = 6 for a ring of 32, 7 for 64,
// where base is wave-uniform and advances by R at every block of R
// positions (all ring keys are rebased by -R there; a live key's offset is
// then at least R, so no borrow reaches the potential).  Offsets of the
// window lie in [0, 2R), so a plain minimum over keys yields the minimum
// potential and, among equal potentials, the smallest p: the evaluator's
// masked window minimum (window_min_asm.inc) runs unchanged on keys.  This
// needs |f| < 2^(29-B), i.e. 3 n maxcost < 2^(29-B) for the tour; feasible
// keys then stay below 2^29 and keys reached only through infeasible
// prefixes (the empty-window sentinel 2^30) stay above it, below 2^31.
// Tours past that bound take the wide path: potentials unpacked and the
// argmin tracked per cell (window_argmin_asm.inc), under the evaluator's
// own guard 3 n maxcost < 2^29.
//
// Layout (position-major, so one wave's stores per position are a single
// 128-byte line):  pred[(i-1)*S + s]  and  cuts[(r-1)*S + s].
//
// Kernels:
//   prep (shared with the evaluator, one tour);
//   routes_key_kernel<R,F,G,E> / routes_wide_kernel<R,F,E>: one wave per
//     tile of 64 scenarios (each returns at once unless the tour takes its
//     path), the tile's demand rows staged in LDS as bytes, pred written per
//     position; then each lane walks its chain back from n (the column it
//     just wrote, still in L2), counting the routes, and walks it again
//     writing the route ends;
//   routes_fallback_kernel: exact recomputation (any window length, any
//     demand value) of the tiles the main kernel listed, then the same
//     backtracking; its last block marks every scenario invalid when the
//     tour or a demand failed validation.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "split_device.h"
#include "split_eval.h"
#include "split_internal.h"

namespace splitk {

namespace {

constexpr int kFeasible = 1 << 29; // m_i below this <=> V(i) finite
constexpr uint16_t kNoPred = 0xFFFF;

#include "window_argmin_asm.inc"
#include "window_min_asm.inc"

template <int R> constexpr int key_shift() { return R == 32 ? 6 : 7; }

// the tour's potentials fit packed keys of shift B
__device__ __forceinline__ bool keys_fit(const TourRec &rec, int B)
{
    return (long long)3 * rec.n * rec.maxc < (1LL << (29 - B));
}

// Backtracking of one scenario from position n.  pcol / ccol point at the
// scenario's column of pred / cuts (stride S).  Returns the number of
// routes, or -1 if the chain does not descend (never for a finite V(n)).
__device__ __forceinline__ int backtrack(const uint16_t *pcol, uint16_t *ccol, int64_t S, int n)
{
    int k = 0;
    for (int i = n; i > 0;) {
        const int p = pcol[(int64_t)(i - 1) * S];
        if (p >= i)
            return -1;
        ++k;
        i = p;
    }
    int r = k;
    for (int i = n; i > 0 && r > 0;) {
        ccol[(int64_t)(--r) * S] = (uint16_t)i;
        const int p = pcol[(int64_t)(i - 1) * S];
        if (p >= i)
            break;
        i = p;
    }
    return k;
}

struct RtRegs {
    int L;          // load of positions 1..j (at the start of position j)
    int qa;         // demand of position j+1 (arrived)
    int2 t0, t1, t2; // table entries of positions j, j+1, j+2
    uint64_t cp1;   // lanes rejecting d = F at position j (computed at j-1)
    int mres;       // m of the last position relaxed
    int ovf;        // 1 when a window reached past the ring
    uint16_t *prow; // pred row of position j (wave-uniform), advanced by S
};

template <int R, int F, int E, int U, bool CHK> struct RtState {
    template <class Src>
    __device__ __forceinline__ static bool run(int (&f)[R], int (&lq)[R], RtRegs &r, Src &src,
                                               CInt *tab, int j0, int n, int Q, int64_t S,
                                               int lane)
    {
        const int j = j0 + U;
        if (U == 0 && j == 0)
            return true;
        if (CHK && j > n)
            return false;
        const int cj = r.t0.y;
        const int Ln = r.L + r.qa;
        r.qa = src.template ahead<U>(r.t2);
        const int2 t3 = tab_at(tab, j + 3);
        uint64_t cn1;
        int a;
        const int m = WindowArgmin<R, F, E>::template run<U>(f, lq, r.L, Ln, j, r.cp1, cn1, a,
                                                             r.ovf);
        r.mres = m;
        f[U] = m + cj;
        lq[U] = r.L + Q;
        r.L = Ln;
        r.cp1 = cn1;
        r.t0 = r.t1;
        r.t1 = r.t2;
        r.t2 = t3;
        r.prow[lane] = (uint16_t)(j - a); // +inf positions are marked after the pass
        r.prow += S;
        return true;
    }
};

template <int R, int F, int E, bool CHK, class Src, int... Us>
__device__ __forceinline__ bool rt_block(int (&f)[R], int (&lq)[R], RtRegs &r, Src &src,
                                         CInt *tab, int j0, int n, int Q, int64_t S, int lane,
                                         std::integer_sequence<int, Us...>)
{
    return (RtState<R, F, E, Us, CHK>::run(f, lq, r, src, tab, j0, n, Q, S, lane) && ...);
}

// Writes pred(1..n) of the lane's scenario; returns m_n, sets ovf when a
// window left the ring.  prow0 = pred + s0 (the tile's first column).
template <int R, int F, int E, class Src>
__device__ __forceinline__ int rt_lane(Src &src, CInt *tab, int n, int f0, int Q,
                                       uint16_t *prow0, int64_t S, int lane, bool &ovf)
{
    int f[R], lq[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        f[i] = kInf;
        lq[i] = kNeg;
    }
    f[0] = f0; // p = 0: V(0) + a_1
    lq[0] = Q; // L_0 + Q
    RtRegs r;
    r.mres = kInf;
    r.ovf = 0;
    r.cp1 = ~0ull; // position 1 starts in the masked path
    r.t0 = tab_at(tab, 1);
    r.t1 = tab_at(tab, 2);
    r.t2 = tab_at(tab, 3);
    src.init(r.t0, r.t1, r.L, r.qa);
    r.prow = prow0;
    int j0 = 0;
    for (; j0 + R - 1 <= n; j0 += R) // blocks whose positions all exist
        rt_block<R, F, E, false>(f, lq, r, src, tab, j0, n, Q, S, lane,
                                 std::make_integer_sequence<int, R>{});
    if (j0 <= n) // the last, partial block
        rt_block<R, F, E, true>(f, lq, r, src, tab, j0, n, Q, S, lane,
                                std::make_integer_sequence<int, R>{});
    ovf = r.ovf != 0;
    return r.mres;
}

// ---------------------------------------------------------------------------
// packed-key recursion
// ---------------------------------------------------------------------------
struct RkRegs {
    int L;           // load of positions 1..j (at the start of position j)
    int qa;          // demand of position j+1 (arrived)
    int2 t0, t1, t2; // table entries of positions j, j+1, j+2
    uint64_t cp1;    // lanes rejecting d = F at position j (computed at j-1)
    uint64_t cp2;    // lanes rejecting d = F + G at position j (computed at j-1)
    int mres;        // key minimum of the last position relaxed
    int ovf;         // 1 when a window reached past the ring
    int base;        // key offset origin of the current block (wave-uniform)
    uint16_t *prow;  // pred row of position j (wave-uniform), advanced by S
};

template <int R, int F, int G, int E, int U, bool CHK> struct RkState {
    template <class Src>
    __device__ __forceinline__ static bool run(int (&K)[R], int (&lq)[R], RkRegs &r, Src &src,
                                               CInt *tab, int j0, int n, int Q, int64_t S,
                                               int lane)
    {
        constexpr int B = key_shift<R>();
        constexpr int M = (1 << B) - 1;
        const int j = j0 + U;
        if (CHK && j > n)
            return false;
        if (U == 0) {
            if (j == 0)
                return true;
#pragma unroll
            for (int i = 0; i < R; ++i) // new block: offsets of the live keys drop by R
                K[i] -= R;
            r.base += R;
        }
        const int cj = r.t0.y;
        const int Ln = r.L + r.qa;
        r.qa = src.template ahead<U>(r.t2);
        const int2 t3 = tab_at(tab, j + 3);
        uint64_t cn1, cn2;
        const int km = WindowMin<R, F, G, E>::template run<U>(K, lq, r.L, Ln, j, r.cp1, r.cp2,
                                                              cn1, cn2, r.ovf);
        r.mres = km;
        // K_j = (m + c_j) * 2^B + (j - base), with m * 2^B = km & ~M
        K[U] = (km & ~M) + ((cj << B) + (j - r.base));
        lq[U] = r.L + Q;
        r.L = Ln;
        r.cp1 = cn1;
        r.cp2 = cn2;
        r.t0 = r.t1;
        r.t1 = r.t2;
        r.t2 = t3;
        r.prow[lane] = (uint16_t)(r.base + (km & M)); // +inf positions: marked after the pass
        r.prow += S;
        return true;
    }
};

template <int R, int F, int G, int E, bool CHK, class Src, int... Us>
__device__ __forceinline__ bool rk_block(int (&K)[R], int (&lq)[R], RkRegs &r, Src &src,
                                         CInt *tab, int j0, int n, int Q, int64_t S, int lane,
                                         std::integer_sequence<int, Us...>)
{
    return (RkState<R, F, G, E, Us, CHK>::run(K, lq, r, src, tab, j0, n, Q, S, lane) && ...);
}

// Writes pred(1..n) of the lane's scenario; returns V(n) (kInf if +inf),
// sets ovf when a window left the ring.
template <int R, int F, int G, int E, class Src>
__device__ __forceinline__ int rk_lane(Src &src, CInt *tab, const TourRec &rec, int Q,
                                       uint16_t *prow0, int64_t S, int lane, bool &ovf)
{
    constexpr int B = key_shift<R>();
    int K[R], lq[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        K[i] = kInf;
        lq[i] = kNeg;
    }
    RkRegs r;
    r.base = -R;
    K[0] = (rec.f0 << B) + (0 - r.base); // p = 0: V(0) + a_1
    lq[0] = Q;                           // L_0 + Q
    r.mres = kInf;
    r.ovf = 0;
    r.cp1 = ~0ull; // position 1 starts in the tail
    r.cp2 = ~0ull;
    r.t0 = tab_at(tab, 1);
    r.t1 = tab_at(tab, 2);
    r.t2 = tab_at(tab, 3);
    src.init(r.t0, r.t1, r.L, r.qa);
    r.prow = prow0;
    const int n = rec.n;
    int j0 = 0;
    for (; j0 + R - 1 <= n; j0 += R) // blocks whose positions all exist
        rk_block<R, F, G, E, false>(K, lq, r, src, tab, j0, n, Q, S, lane,
                                    std::make_integer_sequence<int, R>{});
    if (j0 <= n) // the last, partial block
        rk_block<R, F, G, E, true>(K, lq, r, src, tab, j0, n, Q, S, lane,
                                   std::make_integer_sequence<int, R>{});
    ovf = r.ovf != 0;
    return r.mres < kFeasible ? (r.mres >> B) + rec.bn : kInf;
}

// Backtracking of a tile after the recursion, with one walk per lane: the
// chain is followed through the pred column the lane just wrote (still in
// L2), each route end is marked in a bitmask in LDS ([W][64] words, W =
// ceil(n/32); the demand bytes are dead by then), and a scan of the bitmask
// in increasing position writes the cut points in order, so the number of
// routes need not be known before the first one is written.  Each lane
// reads and writes only its own LDS column.  Returns the number of routes
// of the lane (0 if `chain` is false, -1 if the chain does not descend,
// which a finite V(n) excludes).
__device__ __forceinline__ int lds_words(int n) { return (n + 31) >> 5; }

__device__ __forceinline__ int backtrack_tile(const uint16_t *pcol, uint16_t *ccol, int64_t S,
                                              int n, int lane, bool chain, uint8_t *lds)
{
    const int W = lds_words(n);
    uint32_t *bits = reinterpret_cast<uint32_t *>(lds) + lane;
    for (int w = 0; w < W; ++w)
        bits[w * kWave] = 0;
    if (!chain)
        return 0;
    for (int i = n; i > 0;) {
        bits[((i - 1) >> 5) * kWave] |= 1u << ((i - 1) & 31);
        const int p = pcol[(int64_t)(i - 1) * S];
        if (p >= i)
            return -1;
        i = p;
    }
    int r = 0;
    for (int w = 0; w < W; ++w) {
        uint32_t word = bits[w * kWave];
        while (word) {
            const int b = __builtin_ctz(word);
            word &= word - 1;
            ccol[(int64_t)(r++) * S] = (uint16_t)(32 * w + b + 1);
        }
    }
    return r;
}

// V(n) of the lane's scenario (kInf if +inf) with pred(1..n) written, by
// packed keys (KEYS) or the per-cell argmin.  The recursion stores every
// position's predecessor without testing it; V(j) is +inf exactly from the
// first position whose demand alone exceeds Q (its window is empty, and
// every later window lies past it), so a scenario with V(n) = +inf gets
// SPLIT_NO_PRED from that position on here, off the per-position path.
template <bool KEYS, int R, int F, int G, int E, class Src>
__device__ __forceinline__ int route_lane(Src &src, CInt *tab, const TourRec &rec, int Q,
                                          uint16_t *prow0, int64_t S, int lane, bool &ovf)
{
    int v;
    if constexpr (KEYS) {
        v = rk_lane<R, F, G, E>(src, tab, rec, Q, prow0, S, lane, ovf);
    } else {
        const int m = rt_lane<R, F, E>(src, tab, rec.n, rec.f0, Q, prow0, S, lane, ovf);
        v = m < kFeasible ? m + rec.bn : kInf;
    }
    if (v >= kInf) {
        int j = 1;
        while (j <= rec.n && src.at(tab, j) <= Q)
            ++j;
        for (; j <= rec.n; ++j)
            prow0[(int64_t)(j - 1) * S + lane] = kNoPred;
    }
    return v;
}

// Tile body shared by the key and the wide kernel: stage the tile (or, ORD,
// read the tour-ordered copy the permute kernel wrote), run the lane
// recursion, backtrack, or list the tile for the exact fallback.
// KEYS: packed keys with ring R and window variant (F, G, E); otherwise the
// per-cell argmin with ring R and (F, E), serving the tours whose costs are
// too wide for keys of key_bits.
template <bool KEYS, bool ORD, int R, int F, int G, int E>
__device__ __forceinline__ void routes_tile(const int16_t *__restrict__ demands, int32_t N,
                                            int64_t S, int32_t Q, int32_t *__restrict__ costs,
                                            uint16_t *pred, uint16_t *cuts,
                                            int32_t *__restrict__ nroutes, const Workspace &ws,
                                            int32_t lds_bytes, int32_t pitch, const int2 *tabp,
                                            int key_bits)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const TourRec rec = ws.rec[0];
    if (rec.status != ST_OK)
        return; // the fallback kernel's last block marks every scenario
    if (keys_fit(rec, key_bits) != KEYS)
        return; // the other kernel serves this tour
    const int64_t k = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t s0 = k * kWave;
    const int rows = (int)min<int64_t>(kWave, S - s0);
    if (rec.n == 0) {
        if (lane < rows) {
            costs[s0 + lane] = 0;
            nroutes[s0 + lane] = 0;
        }
        return;
    }
    bool ok = false;
    CInt *tab;
    if constexpr (ORD) {
        // the permute kernel flagged tiles with a demand outside [0, 255]
        ok = ws.tile_bad[k] == 0;
        tab = (CInt *)ws.tab;
    } else {
        // whole scenario rows (pitch 0: row stride N, indexed by customer) or
        // the tour's demands gathered in tour order (row stride pitch, by
        // position)
        const int stride = pitch ? pitch : N;
        if (lds_bytes) {
            int &s_bad =
                *reinterpret_cast<int *>(lds + (((size_t)kWave * stride + 15) & ~(size_t)15));
            ok = pitch ? stage_tile_gather_u8(demands + s0 * N, N, rows, ws.tab, rec.n, pitch, lds,
                                              lane, kWave, s_bad)
                       : stage_tile_u8(demands + s0 * N, lds, (int64_t)rows * N, lane, kWave,
                                       s_bad);
        }
        tab = (CInt *)(pitch ? tabp : ws.tab);
    }
    bool redo = true;
    if (ok) {
        bool ovf = false;
        int v = kInf;
        if (lane < rows) {
            if constexpr (ORD) {
                StreamRow src;
                src.row = reinterpret_cast<const u32x4 *>(ws.perm + (s0 + lane) * (int64_t)pitch);
                src.segs = pitch / 32;
                v = route_lane<KEYS, R, F, G, E>(src, tab, rec, Q, pred + s0, S, lane, ovf);
            } else {
                LdsRow src{lds + (int64_t)lane * (pitch ? pitch : N)};
                v = route_lane<KEYS, R, F, G, E>(src, tab, rec, Q, pred + s0, S, lane, ovf);
            }
        }
        redo = ballot(ovf) != 0;
        if (!redo) {
            const int64_t s = s0 + lane;
            const bool live = lane < rows, fin = v < kInf;
            if (live)
                costs[s] = fin ? v : SPLIT_INF;
            if (live) {
                int nr = 0;
                if (lds_words(rec.n) * 4 * kWave <= lds_bytes)
                    nr = backtrack_tile(pred + s, cuts + s, S, rec.n, lane, fin, lds);
                else if (fin)
                    nr = backtrack(pred + s, cuts + s, S, rec.n);
                nroutes[s] = nr;
            }
        }
    }
    if (redo && lane == 0) {
        const int slot = atomicAdd(ws.list_count, 1);
        ws.list[slot] = (int)k;
    }
}

// grid = tiles, one wave each; LDS: the demand tile + flag word (or, ORD,
// only the backtracking bitmask; pitch is then the ordered copy's row
// stride).  Serves tours whose potentials fit packed keys of this ring.
template <int R, int F, int G, int E, bool ORD>
__global__ __launch_bounds__(kWave) void routes_key_kernel(
    const int16_t *__restrict__ demands, int32_t N, int64_t S, int32_t Q,
    int32_t *__restrict__ costs, uint16_t *pred, uint16_t *cuts, int32_t *__restrict__ nroutes,
    Workspace ws, int32_t lds_bytes, int32_t pitch, const int2 *tabp)
{
    routes_tile<true, ORD, R, F, G, E>(demands, N, S, Q, costs, pred, cuts, nroutes, ws,
                                       lds_bytes, pitch, tabp, key_shift<R>());
}

// Same grid and LDS; serves the tours that keys of key_bits cannot hold.
template <int R, int F, int E, bool ORD>
__global__ __launch_bounds__(kWave) void routes_wide_kernel(
    const int16_t *__restrict__ demands, int32_t N, int64_t S, int32_t Q,
    int32_t *__restrict__ costs, uint16_t *pred, uint16_t *cuts, int32_t *__restrict__ nroutes,
    Workspace ws, int32_t lds_bytes, int32_t pitch, const int2 *tabp, int32_t key_bits)
{
    routes_tile<false, ORD, R, F, 0, E>(demands, N, S, Q, costs, pred, cuts, nroutes, ws,
                                        lds_bytes, pitch, tabp, key_bits);
}

// grid = kFallbackBlocks waves; exact recursion for listed tiles with
// the value history in workspace scratch ([j][lane] per block)
__global__ __launch_bounds__(kWave) void routes_fallback_kernel(
    const int16_t *__restrict__ demands, int32_t N, int64_t S, int32_t Q, int32_t *costs,
    uint16_t *pred, uint16_t *cuts, int32_t *nroutes, Workspace ws)
{
    const int lane = threadIdx.x;
    const int count = *ws.list_count;
    int *V = ws.vscratch + (int64_t)blockIdx.x * kWave * (ws.max_len + 1);
    const TourRec rec = ws.rec[0];
    const int n = rec.n;
    const int2 *tab = ws.tab;
    const int2 *ab = ws.ab;
    for (int li = blockIdx.x; li < count && rec.status == ST_OK; li += gridDim.x) {
        const int64_t k = ws.list[li];
        const int64_t s0 = k * kWave;
        const int rows = (int)min<int64_t>(kWave, S - s0);
        bool negq = false;
        if (lane < rows) {
            const int64_t s = s0 + lane;
            const int16_t *qrow = demands + s * N;
            V[lane] = 0; // V(0)
            for (int j = 1; j <= n; ++j) {
                const int bj = ab[j - 1].y;
                int best = kInf, arg = -1, load = 0;
                for (int p = j - 1; p >= 0; --p) { // p decreasing: "<=" keeps the smallest
                    const int q = qrow[tab[p + 1].x];
                    negq = negq || q < 0;
                    load += q;
                    if (load > Q)
                        break;
                    const int vp = V[(int64_t)p * kWave + lane];
                    if (vp < kInf) {
                        const int c = vp + ab[p].x + bj;
                        if (c <= best) {
                            best = c;
                            arg = p;
                        }
                    }
                }
                V[(int64_t)j * kWave + lane] = best;
                pred[(int64_t)(j - 1) * S + s] = arg < 0 ? kNoPred : (uint16_t)arg;
            }
            const int v = V[(int64_t)n * kWave + lane];
            if (v < kInf) {
                costs[s] = v;
                nroutes[s] = backtrack(pred + s, cuts + s, S, n);
            } else {
                costs[s] = SPLIT_INF;
                nroutes[s] = 0;
            }
        }
        if (ballot(negq) != 0 && lane == 0)
            atomicOr(&ws.rec[0].status, ST_BAD_DEMAND);
    }

    int last = 0;
    if (lane == 0) {
        __threadfence();
        last = atomicAdd(ws.done, 1) == (int)gridDim.x - 1;
    }
    last = __shfl(last, 0, kWave);
    if (!last)
        return;
    __threadfence();
    const int status =
        __hip_atomic_load(&ws.rec[0].status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (status == ST_OK)
        return;
    for (int64_t s = lane; s < S; s += kWave) {
        costs[s] = SPLIT_INF;
        nroutes[s] = -1;
    }
}

// Packed-key variants compiled in (each a window variant of the evaluator),
// and the wide-path argmin variant that backs each ring length.
#define SPLIT_ROUTE_KEY_VARIANTS(X) X(32, 6, 3, 3) X(32, 8, 3, 3) X(32, 8, 0, 4) X(64, 16, 4, 4)

template <int R> struct WideOf;
template <> struct WideOf<32> {
    static constexpr int F = 6, E = 3;
};
template <> struct WideOf<64> {
    static constexpr int F = 12, E = 4;
};

// ring length by capacity (longer windows for larger Q); head and exit
// spacing from measured sweeps at n=200, S=10^6 (Q = 80, 150, 300)
RouteVariant default_route_variant(int32_t Q)
{
    if (Q > 200)
        return RouteVariant{64, 16, 4, 4};
    return RouteVariant{32, 8, 0, 4};
}

RouteVariant g_route_override = {0, 0, 0, 0};

// Allows a kernel the LDS limit of the device once; returns that limit.
hipError_t allow_lds(const void *kernel, int *limit)
{
    int dev = 0, lim = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess)
        return e;
    lim = lim < kLdsLimit ? lim : kLdsLimit;
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e == hipSuccess)
        *limit = lim;
    return e;
}

template <int R, int F, int G, int E, bool ORD> struct RouteKernels {
    static constexpr int WF = WideOf<R>::F, WE = WideOf<R>::E;
    // the LDS limit both kernels were allowed (-1 before the first call)
    static hipError_t limit(int *lim)
    {
        static int lim_key = -1, lim_wide = -1;
        hipError_t e = hipSuccess;
        if (lim_key < 0)
            e = allow_lds(reinterpret_cast<const void *>(&routes_key_kernel<R, F, G, E, ORD>),
                          &lim_key);
        if (e == hipSuccess && lim_wide < 0)
            e = allow_lds(reinterpret_cast<const void *>(&routes_wide_kernel<R, WF, WE, ORD>),
                          &lim_wide);
        *lim = lim_key < lim_wide ? lim_key : lim_wide;
        return e;
    }
    static hipError_t launch(const int16_t *demands, int32_t N, int64_t S, int32_t Q,
                             int32_t *costs, uint16_t *pred, uint16_t *cuts, int32_t *nroutes,
                             const Workspace &ws, int32_t lds_bytes, int32_t pitch,
                             const int2 *tabp, hipStream_t stream)
    {
        const dim3 grid((unsigned)num_tiles(S));
        hipLaunchKernelGGL((routes_key_kernel<R, F, G, E, ORD>), grid, dim3(kWave),
                           (size_t)lds_bytes, stream, demands, N, S, Q, costs, pred, cuts,
                           nroutes, ws, lds_bytes, pitch, tabp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL((routes_wide_kernel<R, WF, WE, ORD>), grid, dim3(kWave),
                           (size_t)lds_bytes, stream, demands, N, S, Q, costs, pred, cuts,
                           nroutes, ws, lds_bytes, pitch, tabp, (int32_t)key_shift<R>());
        return hipGetLastError();
    }
};

// Launches the key kernel and the wide kernel of ring R (the one that does
// not serve the tour returns at once): on the demand tile in LDS, or, when
// the workspace holds the tour-ordered copy, after the permute kernel wrote
// it.
template <int R, int F, int G, int E>
hipError_t launch_route_tiles(int32_t n, const int16_t *demands, int32_t N, int64_t S,
                              int32_t Q, int32_t *costs, uint16_t *pred, uint16_t *cuts,
                              int32_t *nroutes, const Workspace &ws, int2 *tabp,
                              hipStream_t stream)
{
    const size_t bits = (size_t)((n + 31) / 32) * 4 * kTile; // backtracking bitmask
    int lim = 0;
    if (ws.perm) {
        hipError_t e = RouteKernels<R, F, G, E, true>::limit(&lim);
        if (e == hipSuccess)
            e = launch_permute(demands, N, S, 1, n, ws, stream);
        if (e != hipSuccess)
            return e;
        const int32_t lds_bytes = bits <= (size_t)lim ? (int32_t)bits : 0;
        return RouteKernels<R, F, G, E, true>::launch(demands, N, S, Q, costs, pred, cuts, nroutes,
                                                      ws, lds_bytes, ordered_pitch(n), tabp,
                                                      stream);
    }
    hipError_t e = RouteKernels<R, F, G, E, false>::limit(&lim);
    if (e != hipSuccess)
        return e;
    // demand tile (whole rows, or the tour gathered) + flag word, and at
    // least room for the backtracking bitmask
    const int32_t pitch = gather_tile(n, N, lim) ? n + 1 : 0;
    const size_t stride = pitch ? (size_t)pitch : (size_t)N;
    const size_t tile = (((size_t)kTile * stride + 15) & ~(size_t)15) + 16;
    const size_t lds = tile > bits ? tile : bits;
    const int32_t lds_bytes = lds <= (size_t)lim ? (int32_t)lds : 0;
    if (pitch && lds_bytes) {
        hipLaunchKernelGGL(position_table_kernel, dim3(1), dim3(256), 0, stream, ws.tab, n, tabp);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return RouteKernels<R, F, G, E, false>::launch(demands, N, S, Q, costs, pred, cuts, nroutes,
                                                   ws, lds_bytes, pitch, tabp, stream);
}

} // namespace

bool route_variant_supported(const RouteVariant &v)
{
#define SPLIT_RV_SUPPORTED(R_, F_, G_, E_)                                                       \
    if (v.ring == R_ && v.first == F_ && v.group == G_ && v.every == E_)                         \
        return true;
    SPLIT_ROUTE_KEY_VARIANTS(SPLIT_RV_SUPPORTED)
#undef SPLIT_RV_SUPPORTED
    return false;
}

int compiled_route_variants(RouteVariant *out, int cap)
{
    int n = 0;
#define SPLIT_RV_LIST(R_, F_, G_, E_)                                                            \
    if (n < cap)                                                                                 \
        out[n] = RouteVariant{R_, F_, G_, E_};                                                   \
    ++n;
    SPLIT_ROUTE_KEY_VARIANTS(SPLIT_RV_LIST)
#undef SPLIT_RV_LIST
    return n;
}

RouteVariant choose_route_variant(int32_t Q)
{
    return g_route_override.ring ? g_route_override : default_route_variant(Q);
}

static size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

static int g_route_path = 0; // 0 automatic, 1 demand tile in LDS, 2 tour-ordered copy

void set_route_path(int path) { g_route_path = path; }

// Whole-row tiles above this many bytes per wave stream the tour-ordered
// copy instead (measured at n = N: 300 is faster in LDS, 500 streamed).
constexpr int64_t kRouteTileMax = 24 * 1024;

bool routes_ordered(int32_t n, int32_t N)
{
    if (n == 0 || !ordered_path_possible(N, n))
        return false;
    if (g_route_path)
        return g_route_path == 2;
    // a tour over at most half of the pool would be gathered into LDS with
    // scattered 2-byte loads; the permute kernel's coalesced row reads and
    // the streamed copy measured faster there (n = 200, N = 1000)
    const bool gathered = 2 * ((int64_t)n + 1) <= N;
    return gathered || (int64_t)kTile * N > kRouteTileMax;
}

size_t routes_workspace_bytes(int32_t n, int32_t N, int64_t S)
{
    // the evaluator's one-tour workspace (with the tour-ordered copy when
    // that path is taken), then the position table of a gathered tile
    return round256(workspace_bytes(1, n, N, S, routes_ordered(n, N))) +
           round256(((size_t)n + kTabPad) * sizeof(int2));
}

int2 *routes_position_table(void *workspace, int32_t n, int32_t N, int64_t S)
{
    return reinterpret_cast<int2 *>(static_cast<char *>(workspace) +
                                    round256(workspace_bytes(1, n, N, S, routes_ordered(n, N))));
}

hipError_t launch_routes(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                         const int16_t *demands, int64_t S, int32_t Q, int32_t *costs,
                         uint16_t *pred, uint16_t *cuts, int32_t *nroutes, const Workspace &ws,
                         int2 *tabp, hipStream_t stream, const RouteVariant &v,
                         const LaunchEvents *ev)
{
    if (!route_variant_supported(v))
        return hipErrorInvalidValue;
    hipError_t e = launch_prep(tour, nullptr, 1, n, dist, N, ws, stream);
    if (e != hipSuccess)
        return e;
    if (ev && ev->before) {
        e = hipEventRecord(ev->before, stream);
        if (e != hipSuccess)
            return e;
    }
#define SPLIT_RV_LAUNCH(R_, F_, G_, E_)                                                          \
    if (v.ring == R_ && v.first == F_ && v.group == G_ && v.every == E_)                         \
        e = launch_route_tiles<R_, F_, G_, E_>(n, demands, N, S, Q, costs, pred, cuts, nroutes,  \
                                               ws, tabp, stream);
    SPLIT_ROUTE_KEY_VARIANTS(SPLIT_RV_LAUNCH)
#undef SPLIT_RV_LAUNCH
    if (e != hipSuccess)
        return e;
    if (ev && ev->after) {
        e = hipEventRecord(ev->after, stream);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(routes_fallback_kernel, dim3(kFallbackBlocks), dim3(kWave), 0, stream,
                       demands, N, S, Q, costs, pred, cuts, nroutes, ws);
    return hipGetLastError();
}

void set_route_override(const RouteVariant &v) { g_route_override = v; }

} // namespace splitk
