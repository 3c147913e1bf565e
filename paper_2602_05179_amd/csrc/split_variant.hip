// split_variant.hip -- split variants from the extensive form's objective
// and constraints (App. A): soft capacity, where each route pays
// beta * max(0, load - Q) instead of being excluded (the per-vehicle
// overload term), and a fleet of at most K routes (the fleet-size bound).
//
// With J_k(i) the cheapest split of positions 1..i into exactly k routes,
//   J_0(0) = 0, J_0(i > 0) = +inf,  J_k(i) = min_{p<i} J_{k-1}(p) + cost(p,i),
// the scenario's cost is min_{k<=K} J_k(n); K = 0 is the unlimited fleet,
// J(i) = min_{p<i} J(p) + cost(p,i).  beta < 0 keeps the hard capacity.
//
// Potential form as in split_kernels.hip: f_p = J(p) + a_{p+1},
// J(i) = b_i + min_p (f_p + beta * max(0, L_i - (L_p + Q))), so a ring cell
// costs its potential plus the penalty of its overload, and the next
// potential is m_i + c_i.  Soft capacity: every predecessor is admissible,
// so besides the R ring cells the scan needs the cells that have left the
// ring; a cell leaves the ring R positions after it entered, and if it is
// then outside the hard window [p_min(i), i-1] it stays overloaded for every
// later position (loads only grow), with cost (f_p - beta (L_p + Q)) +
// beta L_i: those fold into one running minimum per lane.  A lane whose
// hard window reaches R cells (it admits d = R while i > R) would break
// that argument, and its tile goes to the exact fallback, as in the
// evaluator.  Fleet bound: K passes over the tour inside the kernel; pass
// k streams the potentials of pass k-1 from a position-major buffer in the
// workspace into its ring and writes its own.
//
// Ranges: potentials are clamped at the 2^30 sentinel after every position,
// so values descending from +inf stay in [2^30 - maxcost, 2^30 + 2 maxcost
// + beta (L_n + Q)] while feasible ones stay below 2^29 when
// 3 n maxcost + beta (L_n + Q) < 2^29 and L_n + Q < 2^24 (the penalty is
// a 24-bit multiply).  The recursion checks that per scenario and flags
// the call (status bit ST_PENALTY_RANGE) otherwise.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "split_device.h"
#include "split_eval.h"
#include "split_internal.h"
#include "split_variant.h"

namespace splitk {

namespace {

constexpr int kFeasible = 1 << 29;
constexpr int ST_PENALTY_RANGE = 4;

#include "window_min_asm.inc"
#include "window_min_multi_asm.inc"

// hard capacity: the evaluator's window variant for each ring length
template <int R> struct HardWindow;
template <> struct HardWindow<32> {
    static constexpr int F = 8, G = 3, E = 3;
};
template <> struct HardWindow<64> {
    static constexpr int F = 16, G = 4, E = 4;
};

struct VarArgs {
    const int16_t *demands;
    int32_t N;
    int64_t S;
    int32_t Q;
    int32_t beta; // < 0: hard capacity
    int32_t K;    // 0: unlimited fleet
    int32_t *costs;
    int *lay0, *lay1; // [n][S] potentials of consecutive passes (K > 0)
    int *vs;          // fallback scratch [blocks][2][n+1][64]
    int32_t pitch;    // 0: whole scenario rows in LDS; else the tour gathered, row stride pitch
    const int2 *tabp; // per-tour table indexed by position (gathered tile)
    int32_t opitch;   // row stride of the tour-ordered copy (ordered kernels)
};

// Stages the tile (whole rows or the tour gathered) and returns the table
// and row stride the recursion reads it with.
__device__ __forceinline__ bool stage_variant_tile(const VarArgs &a, const Workspace &ws, int n,
                                                   int64_t s0, int rows, uint8_t *lds, int lane,
                                                   CInt *&tab, int &stride)
{
    stride = a.pitch ? a.pitch : a.N;
    tab = (CInt *)(a.pitch ? a.tabp : ws.tab);
    int &s_bad = *reinterpret_cast<int *>(lds + (((size_t)kWave * stride + 15) & ~(size_t)15));
    return a.pitch ? stage_tile_gather_u8(a.demands + s0 * a.N, a.N, rows, ws.tab, n, a.pitch, lds,
                                          lane, kWave, s_bad)
                   : stage_tile_u8(a.demands + s0 * a.N, lds, (int64_t)rows * a.N, lane, kWave,
                                   s_bad);
}

struct VarRegs {
    int L;           // load of positions 1..j
    int qa;          // demand of position j+1
    int2 t0, t1, t2; // table entries of positions j, j+1, j+2
    int pf0, pf1;    // previous pass's potentials of positions j, j+1 (layered)
    int mret;        // soft: min over retired cells of f_p - beta (L_p + Q)
    int mres;        // m of the last position relaxed
    int lastL;       // load of positions 1..n (set at position n)
    int ovf;
    uint64_t cp1, cp2; // hard capacity: lanes rejecting the head groups at j
    const int *srcp; // previous pass, row j+2 of this lane's column (layered)
    int *dstp;       // this pass, row j (layered)
};

// One position j = j0 + U.  LAYERED: the ring holds the previous pass's
// potentials and this pass's are written out; otherwise the ring holds the
// pass's own potentials (unlimited fleet).
template <int R, bool SOFT, bool LAYERED, int U, bool CHK> struct VarState {
    template <class Src>
    __device__ __forceinline__ static bool run(int (&f)[R], int (&lq)[R], VarRegs &r, Src &src,
                                               CInt *tab, int j0, int n, int Q, int beta,
                                               bool has_src, int64_t S)
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
        int pf2 = kInf;
        if constexpr (LAYERED) {
            if (has_src) { // uniform: the first pass has no previous potentials
                if (j + 2 <= n - 1)
                    pf2 = *r.srcp;
                r.srcp += S;
            }
        }
        const int L = r.L;
        if (j == n)
            r.lastL = L;
        int m = kInf;
        if constexpr (SOFT) {
            // every ring cell, each with the penalty of its overload
#pragma unroll
            for (int d = 1; d <= R; ++d) {
                const int fd = f[(U - d) & (R - 1)];
                // max(L - lq, 0) as one clamped unsigned subtract (L, lq >= 0)
                const unsigned t =
                    __builtin_elementwise_sub_sat((unsigned)L, (unsigned)lq[(U - d) & (R - 1)]);
                m = min(m, fd + (int)__umul24((unsigned)beta, t));
            }
            m = min(m, r.mret + (int)__umul24((unsigned)beta, (unsigned)L));
            // the cell leaving the ring (p = j - R) sits in slot U
            if (j > R && L <= lq[U])
                r.ovf = 1;
        } else {
            // the admissible window only (sets ovf itself)
            using HW = HardWindow<R>;
            uint64_t cn1, cn2;
            m = WindowMin<R, HW::F, HW::G, HW::E>::template run<U>(f, lq, L, Ln, j, r.cp1,
                                                                   r.cp2, cn1, cn2, r.ovf);
            r.cp1 = cn1;
            r.cp2 = cn2;
        }
        m = min(m, kInf);
        r.mres = m;
        if constexpr (SOFT) {
            if (j >= R) // slot U holds p = j - R >= 0
                r.mret = min(r.mret, f[U] - (int)__umul24((unsigned)beta, (unsigned)lq[U]));
        }
        const int fj = m + cj;
        if constexpr (LAYERED) {
            if (j <= n - 1)
                *r.dstp = fj;
            r.dstp += S;
            f[U] = r.pf0; // previous pass's potential of p = j
            r.pf0 = r.pf1;
            r.pf1 = pf2;
        } else {
            f[U] = fj;
        }
        lq[U] = L + Q;
        r.L = Ln;
        r.t0 = r.t1;
        r.t1 = r.t2;
        r.t2 = t3;
        return true;
    }
};

template <int R, bool SOFT, bool LAYERED, bool CHK, class Src, int... Us>
__device__ __forceinline__ bool var_block(int (&f)[R], int (&lq)[R], VarRegs &r, Src &src,
                                          CInt *tab, int j0, int n, int Q, int beta, bool has_src,
                                          int64_t S, std::integer_sequence<int, Us...>)
{
    return (VarState<R, SOFT, LAYERED, Us, CHK>::run(f, lq, r, src, tab, j0, n, Q, beta, has_src, S) &&
            ...);
}

// One pass over the tour, reading the demands from a fresh copy of dsrc.
// src: previous pass's potentials of this lane's column (nullptr for the
// first pass of a layered run); dst: this pass's.  Returns m_n.
template <int R, bool SOFT, bool LAYERED, class Src>
__device__ __forceinline__ int var_pass(Src dsrc, CInt *tab, const TourRec &rec, int Q, int beta,
                                        int first_f, const int *src, int *dst, int64_t S,
                                        bool &ovf, int &Ltot)
{
    // slots before the tour start: potential +inf; soft capacity gives them
    // a threshold no load reaches (cost +inf without a mask), hard capacity
    // one every load exceeds (never admissible)
    int f[R], lq[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        f[i] = kInf;
        lq[i] = SOFT ? kInf : kNeg;
    }
    f[0] = first_f; // p = 0
    lq[0] = Q;
    VarRegs r;
    r.mret = kInf;
    r.mres = kInf;
    r.lastL = 0;
    r.ovf = 0;
    r.cp1 = ~0ull; // position 1 starts in the tail
    r.cp2 = ~0ull;
    r.t0 = tab_at(tab, 1);
    r.t1 = tab_at(tab, 2);
    r.t2 = tab_at(tab, 3);
    dsrc.init(r.t0, r.t1, r.L, r.qa);
    const int n = rec.n;
    r.pf0 = kInf;
    r.pf1 = kInf;
    r.srcp = nullptr;
    r.dstp = nullptr;
    const bool has_src = src != nullptr;
    if constexpr (LAYERED) {
        if (has_src) {
            if (n >= 2)
                r.pf0 = src[S];
            if (n >= 3)
                r.pf1 = src[2 * S];
            r.srcp = src + 3 * S; // row j+2 at position j = 1
        }
        r.dstp = dst + S; // row j at position j = 1
    }
    int j0 = 0;
    for (; j0 + R - 1 <= n; j0 += R) // blocks whose positions all exist
        var_block<R, SOFT, LAYERED, false>(f, lq, r, dsrc, tab, j0, n, Q, beta, has_src, S,
                                           std::make_integer_sequence<int, R>{});
    if (j0 <= n) // the last, partial block
        var_block<R, SOFT, LAYERED, true>(f, lq, r, dsrc, tab, j0, n, Q, beta, has_src, S,
                                          std::make_integer_sequence<int, R>{});
    ovf = r.ovf != 0;
    Ltot = r.lastL;
    return r.mres;
}

__device__ __forceinline__ bool penalty_fits(const TourRec &rec, int beta, int Q, int Ltot);

// ---------------------------------------------------------------------------
// fleet bound: NL passes per sweep over the tour.  Every pass
// relaxes the same admissible window (it depends on loads only), so one
// masked scan (window_min_multi_asm.inc) serves NL potential rings: ring 0
// holds the previous sweep's last pass (streamed from the workspace), ring
// g the potentials that ring g-1 produces in this sweep, and only the last
// ring's potentials are written out for the next sweep.
// ---------------------------------------------------------------------------
template <int NL> struct VarMultiRegs {
    int L, qa;
    int2 t0, t1, t2;
    int pf0, pf1;
    int mres[NL];
    int mret[NL]; // soft: min over retired cells of f_p - beta (L_p + Q), per ring
    int lastL;
    int ovf;
    uint64_t cp1, cp2;
    const int *srcp;
    int *dstp;
};

template <int R, int NL, bool SOFT, int U, bool CHK> struct VarMultiState {
    template <class Src>
    __device__ __forceinline__ static bool run(int (&f)[NL][R], int (&lq)[R], VarMultiRegs<NL> &r,
                                               Src &src, CInt *tab, int j0, int n, int Q, int beta,
                                               bool has_src, int64_t S)
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
        int pf2 = kInf;
        if (has_src) {
            if (j + 2 <= n - 1)
                pf2 = *r.srcp;
            r.srcp += S;
        }
        const int L = r.L;
        if (j == n)
            r.lastL = L;
        int m[NL];
        if constexpr (SOFT) {
            // the penalty of a cell is the same for every pass: once per cell
#pragma unroll
            for (int g = 0; g < NL; ++g)
                m[g] = r.mret[g] + (int)__umul24((unsigned)beta, (unsigned)L);
#pragma unroll
            for (int d = 1; d <= R; ++d) {
                const int pen = (int)__umul24(
                    (unsigned)beta,
                    __builtin_elementwise_sub_sat((unsigned)L, (unsigned)lq[(U - d) & (R - 1)]));
#pragma unroll
                for (int g = 0; g < NL; ++g)
                    m[g] = min(m[g], f[g][(U - d) & (R - 1)] + pen);
            }
            if (j > R && L <= lq[U])
                r.ovf = 1;
            if (j >= R) { // slot U holds p = j - R >= 0, leaving the ring
                const int bq = (int)__umul24((unsigned)beta, (unsigned)lq[U]);
#pragma unroll
                for (int g = 0; g < NL; ++g)
                    r.mret[g] = min(r.mret[g], f[g][U] - bq);
            }
        } else {
            using HW = HardWindow<R>;
            uint64_t cn1, cn2;
            WindowMinMulti<R, HW::F, HW::G, HW::E, NL>::template run<U>(f, lq, L, Ln, j, r.cp1,
                                                                        r.cp2, cn1, cn2, r.ovf, m);
            r.cp1 = cn1;
            r.cp2 = cn2;
        }
#pragma unroll
        for (int g = 0; g < NL; ++g) {
            m[g] = min(m[g], kInf);
            r.mres[g] = m[g];
        }
        if (j <= n - 1)
            *r.dstp = m[NL - 1] + cj;
        r.dstp += S;
#pragma unroll
        for (int g = NL - 1; g >= 1; --g)
            f[g][U] = m[g - 1] + cj;
        f[0][U] = r.pf0;
        r.pf0 = r.pf1;
        r.pf1 = pf2;
        lq[U] = L + Q;
        r.L = Ln;
        r.t0 = r.t1;
        r.t1 = r.t2;
        r.t2 = t3;
        return true;
    }
};

template <int R, int NL, bool SOFT, bool CHK, class Src, int... Us>
__device__ __forceinline__ bool var_multi_block(int (&f)[NL][R], int (&lq)[R],
                                                VarMultiRegs<NL> &r, Src &src, CInt *tab, int j0,
                                                int n, int Q, int beta, bool has_src, int64_t S,
                                                std::integer_sequence<int, Us...>)
{
    return (VarMultiState<R, NL, SOFT, Us, CHK>::run(f, lq, r, src, tab, j0, n, Q, beta, has_src, S) &&
            ...);
}

// One sweep: passes k0 .. k0+NL-1.  src: pass k0-1's potentials (nullptr
// when k0 = 1); dst: pass k0+NL-1's.  m_n of every pass in mres.
template <int R, int NL, bool SOFT, class Src>
__device__ __forceinline__ void var_sweep(Src dsrc, CInt *tab, const TourRec &rec, int Q, int beta,
                                          int k0, const int *src, int *dst, int64_t S, bool &ovf,
                                          int &Ltot, int (&mres)[NL])
{
    // slots before the tour start: +inf potentials; soft capacity gives them
    // a threshold no load reaches, hard capacity one every load exceeds
    int f[NL][R], lq[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        lq[i] = SOFT ? kInf : kNeg;
#pragma unroll
        for (int g = 0; g < NL; ++g)
            f[g][i] = kInf;
    }
    // p = 0 of pass k0+g-1: V_0(0) = 0 for the pass before the first, +inf after
    f[0][0] = k0 == 1 ? rec.f0 : kInf;
    lq[0] = Q;
    VarMultiRegs<NL> r;
#pragma unroll
    for (int g = 0; g < NL; ++g) {
        r.mres[g] = kInf;
        r.mret[g] = kInf;
    }
    r.lastL = 0;
    r.ovf = 0;
    r.cp1 = ~0ull;
    r.cp2 = ~0ull;
    r.t0 = tab_at(tab, 1);
    r.t1 = tab_at(tab, 2);
    r.t2 = tab_at(tab, 3);
    dsrc.init(r.t0, r.t1, r.L, r.qa);
    const int n = rec.n;
    r.pf0 = kInf;
    r.pf1 = kInf;
    r.srcp = nullptr;
    const bool has_src = src != nullptr;
    if (has_src) {
        if (n >= 2)
            r.pf0 = src[S];
        if (n >= 3)
            r.pf1 = src[2 * S];
        r.srcp = src + 3 * S;
    }
    r.dstp = dst + S;
    // one unrolled copy, bound test at every position: a second (untested)
    // copy of this large block measured slower (three hard rings at n = 200,
    // S = 10^6, K = 25: 5.11 ms vs 4.75 ms)
    for (int j0 = 0; j0 <= n; j0 += R) {
        if (!var_multi_block<R, NL, SOFT, true>(f, lq, r, dsrc, tab, j0, n, Q, beta, has_src,
                                                S, std::make_integer_sequence<int, R>{}))
            break;
    }
    ovf = r.ovf != 0;
    Ltot = r.lastL;
#pragma unroll
    for (int g = 0; g < NL; ++g)
        mres[g] = r.mres[g];
}

// grid = tiles, one wave each; LDS as variant_tile_kernel.  Fleet bound
// K > 0, hard or soft capacity.
// The fleet-bounded passes of one lane, in sweeps of NL: the minimum over
// passes of m_n (kInf if none is finite); sets ovf, Ltot.
template <int R, int NL, bool SOFT, class Src>
__device__ __forceinline__ int multi_lane(const Src &dsrc, CInt *tab, const TourRec &rec,
                                          const VarArgs &a, int64_t s, bool &ovf, int &Ltot)
{
    const int passes = a.K < rec.n ? a.K : rec.n;
    const int *src = nullptr;
    int *dst = a.lay0 + s;
    int best = kInf;
    for (int k0 = 1; k0 <= passes; k0 += NL) {
        bool o = false;
        int mres[NL];
        var_sweep<R, NL, SOFT>(dsrc, tab, rec, a.Q, a.beta, k0, src, dst, a.S, o, Ltot, mres);
        ovf = ovf || o;
#pragma unroll
        for (int g = 0; g < NL; ++g)
            if (k0 + g <= passes)
                best = min(best, mres[g]);
        src = dst;
        dst = (dst == a.lay0 + s) ? a.lay1 + s : a.lay0 + s;
    }
    return best;
}

// The tile's demands: staged in LDS (whole rows or the tour gathered), or,
// ORD, the tour-ordered copy the permute kernel wrote (tiles it flagged
// take the exact fallback).  Returns false when the tile must be redone.
template <bool ORD>
__device__ __forceinline__ bool variant_tile_source(const VarArgs &a, const Workspace &ws,
                                                    const TourRec &rec, int64_t k, int64_t s0,
                                                    int rows, uint8_t *lds, int lane,
                                                    int32_t lds_bytes, CInt *&tab, int &stride)
{
    if constexpr (ORD) {
        tab = (CInt *)ws.tab;
        stride = a.opitch;
        return ws.tile_bad[k] == 0;
    } else {
        tab = nullptr;
        stride = a.N;
        return lds_bytes ? stage_variant_tile(a, ws, rec.n, s0, rows, lds, lane, tab, stride)
                         : false;
    }
}

// grid = tiles, one wave each; LDS as variant_tile_kernel (none when ORD).
// Fleet bound K > 0, hard or soft capacity.
template <int R, int NL, bool SOFT, bool ORD>
__global__ __launch_bounds__(kWave) void variant_multi_kernel(VarArgs a, Workspace ws,
                                                              int32_t lds_bytes)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const TourRec rec = ws.rec[0];
    if (rec.status != ST_OK)
        return;
    const int64_t k = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t s0 = k * kWave;
    const int rows = (int)min<int64_t>(kWave, a.S - s0);
    if (rec.n == 0) {
        if (lane < rows)
            a.costs[s0 + lane] = 0;
        return;
    }
    CInt *tab;
    int stride;
    const bool ok =
        variant_tile_source<ORD>(a, ws, rec, k, s0, rows, lds, lane, lds_bytes, tab, stride);
    bool redo = true;
    if (ok) {
        bool ovf = false, range_bad = false;
        int best = kInf;
        if (lane < rows) {
            const int64_t s = s0 + lane;
            int Ltot = 0;
            if constexpr (ORD) {
                StreamRow src;
                src.row = reinterpret_cast<const u32x4 *>(ws.perm + s * (int64_t)stride);
                src.segs = stride / 32;
                best = multi_lane<R, NL, SOFT>(src, tab, rec, a, s, ovf, Ltot);
            } else {
                const LdsRow src{lds + (int64_t)lane * stride};
                best = multi_lane<R, NL, SOFT>(src, tab, rec, a, s, ovf, Ltot);
            }
            range_bad = !penalty_fits(rec, a.beta, a.Q, Ltot);
        }
        if (ballot(range_bad) != 0 && lane == 0)
            atomicOr(&ws.rec[0].status, ST_PENALTY_RANGE);
        redo = ballot(ovf) != 0;
        if (!redo && lane < rows)
            a.costs[s0 + lane] = best < kFeasible ? best + rec.bn : SPLIT_INF;
    }
    if (redo && lane == 0) {
        const int slot = atomicAdd(ws.list_count, 1);
        ws.list[slot] = (int)k;
    }
}

// the scenario's penalty range fits the int32 and 24-bit arithmetic
__device__ __forceinline__ bool penalty_fits(const TourRec &rec, int beta, int Q, int Ltot)
{
    if (beta < 0)
        return true;
    const long long lq = (long long)Ltot + Q;
    return lq < (1LL << 24) &&
           (long long)3 * rec.n * rec.maxc + (long long)beta * lq < (1LL << 29);
}

// The passes of one lane: one (unlimited fleet) or K (LAYERED); the
// minimum over passes of m_n; sets ovf, Ltot.
template <int R, bool SOFT, bool LAYERED, class Src>
__device__ __forceinline__ int tile_lane(const Src &dsrc, CInt *tab, const TourRec &rec,
                                         const VarArgs &a, int64_t s, bool &ovf, int &Ltot)
{
    if constexpr (!LAYERED) {
        return var_pass<R, SOFT, false>(dsrc, tab, rec, a.Q, a.beta, rec.f0, nullptr, nullptr,
                                        a.S, ovf, Ltot);
    } else {
        const int *src = nullptr;
        int *dst = a.lay0 + s;
        const int passes = a.K < rec.n ? a.K : rec.n;
        int best = kInf;
        for (int kk = 1; kk <= passes; ++kk) {
            bool o = false;
            const int m = var_pass<R, SOFT, true>(dsrc, tab, rec, a.Q, a.beta,
                                                  kk == 1 ? rec.f0 : kInf, src, dst, a.S, o, Ltot);
            ovf = ovf || o;
            best = min(best, m);
            src = dst;
            dst = (dst == a.lay0 + s) ? a.lay1 + s : a.lay0 + s;
        }
        return best;
    }
}

// grid = tiles, one wave each; LDS: the demand tile + flag word (none when
// ORD).  LAYERED: K passes (fleet bound); otherwise one pass (unlimited
// fleet).
template <int R, bool SOFT, bool LAYERED, bool ORD>
__global__ __launch_bounds__(kWave) void variant_tile_kernel(VarArgs a, Workspace ws,
                                                             int32_t lds_bytes)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const TourRec rec = ws.rec[0];
    if (rec.status != ST_OK)
        return;
    const int64_t k = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t s0 = k * kWave;
    const int rows = (int)min<int64_t>(kWave, a.S - s0);
    if (rec.n == 0) {
        if (lane < rows)
            a.costs[s0 + lane] = 0;
        return;
    }
    CInt *tab;
    int stride;
    const bool ok =
        variant_tile_source<ORD>(a, ws, rec, k, s0, rows, lds, lane, lds_bytes, tab, stride);
    bool redo = true;
    if (ok) {
        bool ovf = false, range_bad = false;
        int best = kInf;
        if (lane < rows) {
            const int64_t s = s0 + lane;
            int Ltot = 0;
            if constexpr (ORD) {
                StreamRow src;
                src.row = reinterpret_cast<const u32x4 *>(ws.perm + s * (int64_t)stride);
                src.segs = stride / 32;
                best = tile_lane<R, SOFT, LAYERED>(src, tab, rec, a, s, ovf, Ltot);
            } else {
                const LdsRow src{lds + (int64_t)lane * stride};
                best = tile_lane<R, SOFT, LAYERED>(src, tab, rec, a, s, ovf, Ltot);
            }
            range_bad = !penalty_fits(rec, a.beta, a.Q, Ltot);
        }
        if (ballot(range_bad) != 0 && lane == 0)
            atomicOr(&ws.rec[0].status, ST_PENALTY_RANGE);
        redo = ballot(ovf) != 0;
        if (!redo && lane < rows)
            a.costs[s0 + lane] = best < kFeasible ? best + rec.bn : SPLIT_INF;
    }
    if (redo && lane == 0) {
        const int slot = atomicAdd(ws.list_count, 1);
        ws.list[slot] = (int)k;
    }
}

// Exact recomputation of listed tiles (plain definition, value history in
// scratch), then the last block publishes the status and, if it is not
// clean, marks every scenario SPLIT_INF.
__global__ __launch_bounds__(kWave) void variant_fallback_kernel(VarArgs a, Workspace ws,
                                                                 int32_t *status_out)
{
    const int lane = threadIdx.x;
    const int count = *ws.list_count;
    const TourRec rec = ws.rec[0];
    const int n = rec.n;
    int *Va = a.vs + (int64_t)blockIdx.x * 2 * (n + 1) * kWave;
    int *Vb = Va + (int64_t)(n + 1) * kWave;
    const int2 *tab = ws.tab;
    const int2 *ab = ws.ab;
    const int Q = a.Q, beta = a.beta;
    for (int li = blockIdx.x; li < count && rec.status == ST_OK; li += gridDim.x) {
        const int64_t k = ws.list[li];
        const int64_t s0 = k * kWave;
        const int rows = (int)min<int64_t>(kWave, a.S - s0);
        bool negq = false, range_bad = false;
        if (lane < rows) {
            const int64_t s = s0 + lane;
            const int16_t *qrow = a.demands + s * a.N;
            int Ltot = 0;
            for (int j = 1; j <= n; ++j) {
                const int q = qrow[tab[j].x];
                negq = negq || q < 0;
                Ltot += q;
            }
            range_bad = !penalty_fits(rec, beta, Q, Ltot);
            const bool layered = a.K > 0;
            const int layers = layered ? min(a.K, n) : 1;
            int *prev = Va, *cur = Vb;
            for (int j = 0; j <= n; ++j)
                prev[(int64_t)j * kWave + lane] = j == 0 ? 0 : kInf;
            int best = kInf;
            for (int kk = 1; kk <= layers && !negq && !range_bad; ++kk) {
                int *srcv = layered ? prev : cur;
                cur[lane] = layered ? kInf : 0;
                for (int j = 1; j <= n; ++j) {
                    const int bj = ab[j - 1].y;
                    int bestj = kInf, load = 0;
                    for (int p = j - 1; p >= 0; --p) {
                        load += qrow[tab[p + 1].x];
                        if (beta < 0 && load > Q)
                            break;
                        const int vp = srcv[(int64_t)p * kWave + lane];
                        if (vp >= kInf)
                            continue;
                        int c = vp + ab[p].x + bj;
                        if (beta >= 0 && load > Q)
                            c += beta * (load - Q);
                        bestj = min(bestj, c);
                    }
                    cur[(int64_t)j * kWave + lane] = bestj;
                }
                best = min(best, cur[(int64_t)n * kWave + lane]);
                int *t = prev;
                prev = cur;
                cur = t;
            }
            a.costs[s] = best < kInf ? best : SPLIT_INF;
        }
        if (ballot(negq) != 0 && lane == 0)
            atomicOr(&ws.rec[0].status, ST_BAD_DEMAND);
        if (ballot(range_bad) != 0 && lane == 0)
            atomicOr(&ws.rec[0].status, ST_PENALTY_RANGE);
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
    if (lane == 0)
        *status_out = status;
    if (status == ST_OK)
        return;
    for (int64_t s = lane; s < a.S; s += kWave)
        a.costs[s] = SPLIT_INF;
}

hipError_t allow_lds_once(const void *kernel, int *limit)
{
    if (*limit >= 0)
        return hipSuccess;
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

// LDS of a tile (its row stride set by a.pitch) with the flag word; 0 when
// it does not fit (every tile then takes the exact fallback)
int32_t variant_lds_bytes(const VarArgs &a, int lim)
{
    const size_t stride = a.pitch ? (size_t)a.pitch : (size_t)a.N;
    const size_t lds = (((size_t)kTile * stride + 15) & ~(size_t)15) + 16;
    return lds <= (size_t)lim ? (int32_t)lds : 0;
}

template <int R, bool SOFT, bool LAYERED, bool ORD>
hipError_t launch_variant_tiles_as(const VarArgs &a, const Workspace &ws, hipStream_t stream)
{
    int32_t lds_bytes = 0;
    if constexpr (!ORD) {
        static int lim = -1;
        hipError_t e = allow_lds_once(
            reinterpret_cast<const void *>(&variant_tile_kernel<R, SOFT, LAYERED, false>), &lim);
        if (e != hipSuccess)
            return e;
        lds_bytes = variant_lds_bytes(a, lim);
    }
    hipLaunchKernelGGL((variant_tile_kernel<R, SOFT, LAYERED, ORD>),
                       dim3((unsigned)num_tiles(a.S)), dim3(kWave), (size_t)lds_bytes, stream, a,
                       ws, lds_bytes);
    return hipGetLastError();
}

template <int R, bool SOFT, bool LAYERED>
hipError_t launch_variant_tiles(const VarArgs &a, const Workspace &ws, hipStream_t stream)
{
    return ws.perm ? launch_variant_tiles_as<R, SOFT, LAYERED, true>(a, ws, stream)
                   : launch_variant_tiles_as<R, SOFT, LAYERED, false>(a, ws, stream);
}

template <int R, int NL, bool SOFT, bool ORD>
hipError_t launch_variant_multi_as(const VarArgs &a, const Workspace &ws, hipStream_t stream)
{
    int32_t lds_bytes = 0;
    if constexpr (!ORD) {
        static int lim = -1;
        hipError_t e = allow_lds_once(
            reinterpret_cast<const void *>(&variant_multi_kernel<R, NL, SOFT, false>), &lim);
        if (e != hipSuccess)
            return e;
        lds_bytes = variant_lds_bytes(a, lim);
    }
    hipLaunchKernelGGL((variant_multi_kernel<R, NL, SOFT, ORD>), dim3((unsigned)num_tiles(a.S)),
                       dim3(kWave), (size_t)lds_bytes, stream, a, ws, lds_bytes);
    return hipGetLastError();
}

template <int R, int NL, bool SOFT>
hipError_t launch_variant_multi(const VarArgs &a, const Workspace &ws, hipStream_t stream)
{
    return ws.perm ? launch_variant_multi_as<R, NL, SOFT, true>(a, ws, stream)
                   : launch_variant_multi_as<R, NL, SOFT, false>(a, ws, stream);
}

// passes per sweep of the fleet-bounded kernels: as many rings as keep the
// occupancy the LDS tile allows (3 waves per SIMD at N = 200); the soft
// ring of 64 keeps one pass per sweep
template <int R, bool SOFT> struct SweepRings;
template <> struct SweepRings<32, false> {
    static constexpr int NL = 3;
};
template <> struct SweepRings<64, false> {
    static constexpr int NL = 2;
};
template <> struct SweepRings<32, true> {
    static constexpr int NL = 2;
};

template <int R>
hipError_t launch_variant_ring(const VarArgs &a, const Workspace &ws, hipStream_t stream)
{
    const bool soft = a.beta >= 0, layered = a.K > 0;
    if (!layered)
        return soft ? launch_variant_tiles<R, true, false>(a, ws, stream)
                    : launch_variant_tiles<R, false, false>(a, ws, stream);
    if (!soft)
        return launch_variant_multi<R, SweepRings<R, false>::NL, false>(a, ws, stream);
    if constexpr (R == 32)
        return launch_variant_multi<32, SweepRings<32, true>::NL, true>(a, ws, stream);
    else
        return launch_variant_tiles<R, true, true>(a, ws, stream);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

} // namespace

static int g_variant_path = 0; // 0 automatic, 1 demand tile in LDS, 2 tour-ordered copy

void set_variant_path(int path) { g_variant_path = path; }

// LDS tiles above this many bytes per wave stream the tour-ordered copy
// instead (measured: n = N = 200 faster in LDS, 500 and 1000 streamed).
constexpr int64_t kVariantTileMax = 24 * 1024;

bool variants_ordered(int32_t n, int32_t N, int32_t K)
{
    if (n == 0 || !ordered_path_possible(N, n))
        return false;
    if (g_variant_path)
        return g_variant_path == 2;
    // a tour over at most half of the pool is gathered into LDS; one pass
    // (K = 0) measured faster streamed, but K passes re-read the copy from
    // HBM each sweep and measured faster from the gathered tile (n = 200,
    // N = 1000)
    const bool gathered = 2 * ((int64_t)n + 1) <= N;
    const int64_t tile = (int64_t)kTile * (gathered ? (int64_t)n + 1 : (int64_t)N);
    return tile > kVariantTileMax || (gathered && K == 0);
}

size_t variant_workspace_bytes(int32_t n, int32_t N, int64_t S, int32_t K)
{
    size_t b = align256(workspace_bytes(1, n, N, S, variants_ordered(n, N, K)));
    if (K > 0)
        b += 2 * align256((size_t)n * (size_t)S * sizeof(int));
    b += align256((size_t)kFallbackBlocks * 2 * ((size_t)n + 1) * kWave * sizeof(int));
    b += align256(((size_t)n + kTabPad) * sizeof(int2));
    return b;
}

int variant_ring(int32_t Q) { return Q > 200 ? 64 : 32; }

hipError_t launch_variant(const int32_t *tour, int32_t n, const int32_t *dist, int32_t N,
                          const int16_t *demands, int64_t S, int32_t Q, int32_t beta, int32_t K,
                          int32_t *costs, int32_t *status, void *workspace, hipStream_t stream)
{
    char *p = static_cast<char *>(workspace);
    const bool ordered = variants_ordered(n, N, K);
    const Workspace ws = carve_workspace(p, 1, n, N, S, ordered);
    p += align256(workspace_bytes(1, n, N, S, ordered));
    VarArgs a;
    a.demands = demands;
    a.N = N;
    a.S = S;
    a.Q = Q;
    a.beta = beta < 0 ? -1 : beta;
    a.K = K;
    a.costs = costs;
    a.lay0 = a.lay1 = nullptr;
    if (K > 0) {
        a.lay0 = reinterpret_cast<int *>(p);
        p += align256((size_t)n * (size_t)S * sizeof(int));
        a.lay1 = reinterpret_cast<int *>(p);
        p += align256((size_t)n * (size_t)S * sizeof(int));
    }
    a.vs = reinterpret_cast<int *>(p);
    p += align256((size_t)kFallbackBlocks * 2 * ((size_t)n + 1) * kWave * sizeof(int));
    int2 *tabp = reinterpret_cast<int2 *>(p);
    hipError_t e = launch_prep(tour, nullptr, 1, n, dist, N, ws, stream);
    if (e != hipSuccess)
        return e;
    // a gathered tile when whole rows do not fit or the tour covers at most
    // half of the pool (the LDS limit of the device, as the kernels see it)
    int dev = 0, lim = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess)
        return e;
    lim = lim < kLdsLimit ? lim : kLdsLimit;
    a.pitch = !ordered && gather_tile(n, N, lim) ? n + 1 : 0;
    a.tabp = tabp;
    a.opitch = ordered ? ordered_pitch(n) : 0;
    if (ordered) {
        e = launch_permute(demands, N, S, 1, n, ws, stream);
        if (e != hipSuccess)
            return e;
    }
    if (a.pitch) {
        hipLaunchKernelGGL(position_table_kernel, dim3(1), dim3(256), 0, stream, ws.tab, n, tabp);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    e = variant_ring(Q) == 64 ? launch_variant_ring<64>(a, ws, stream)
                              : launch_variant_ring<32>(a, ws, stream);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(variant_fallback_kernel, dim3(kFallbackBlocks), dim3(kWave), 0, stream, a,
                       ws, status);
    return hipGetLastError();
}

} // namespace splitk
