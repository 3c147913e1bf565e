// split_dp.h -- the per-lane split recursion over a register ring of
// potentials (device code shared by the evaluation kernels and the served
// form's drain kernels; not part of the public ABI).
//
// Potential form (paper Sec. 2.3 recursion): with a_k = c[0][sigma_k] - D_k
// and b_i = D_i + c[sigma_i][0] (D_k the arc length up to position k), every
// route cost is W(p,i) = a_{p+1} + b_i, so V(i) = b_i + m_i with
// m_i = min over the admissible window of f_p = V(p) + a_{p+1}, and the next
// potential is f_i = m_i + c_i with c_i = c[sigma_i][0] + c[0][sigma_{i+1}]
// - c[sigma_i][sigma_{i+1}].  One scenario per lane; the last R potentials
// and thresholds L_p + Q of a lane live in VGPRs, the position loop is
// unrolled R times, and each position's masked window minimum is an
// inline-assembly block of window_min_asm.inc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "split_device.h"

namespace splitk {

// ---------------------------------------------------------------------------
// the per-lane recursion, ring of R potentials in registers
//
// One DpState<...>::run advances every lane of the wave by one tour
// position j (j = R*block + U); ring slot (j - d) mod R = (U - d) mod R holds
// predecessor p = j - d, so every slot is a compile-time register.  Loads
// run one position ahead: while position j is relaxed the demand of j+2 and
// the table entry of j+3 are in flight, and the demand of j+1 has arrived,
// so the load L_{j+1} is known and the next position's head checks are
// issued inside this position's window block.
// ---------------------------------------------------------------------------
#include "window_min_asm.inc"

struct DpRegs {
    int L;       // load of positions 1..j (at the start of position j)
    int qa;      // demand of position j+1 (arrived)
    int2 t0;     // table entry of position j {customer, c}
    int2 t1;     // table entry of position j+1
    int2 t2;     // table entry of position j+2 (in flight)
    uint64_t cp1; // lanes rejecting d = F at position j (computed at j-1)
    uint64_t cp2; // lanes rejecting d = F + G at position j (computed at j-1)
    int mres;     // m of the last position relaxed (m_n after the loop)
    int ovf;      // 1 when a window reached past the ring
};

// CHK: the block may run past position n (the tour's last block); a full
// block skips the per-position bound test
template <int R, int F, int G, int E, int U, bool CHK> struct DpState {
    __device__ __forceinline__ static bool run(int (&f)[R], int (&lq)[R], DpRegs &r,
                                               const uint8_t *row, CInt *tab, int j0, int n,
                                               int Q)
    {
        const int j = j0 + U;
        if (U == 0 && j == 0)
            return true;
        if (CHK && j > n)
            return false;
        const int cj = r.t0.y;
        const int Ln = r.L + r.qa;
        r.qa = row[r.t2.x];
        const int2 t3 = tab_at(tab, j + 3);
        uint64_t cn1, cn2;
        const int m = WindowMin<R, F, G, E>::template run<U>(f, lq, r.L, Ln, j, r.cp1, r.cp2, cn1,
                                                             cn2, r.ovf);
        r.mres = m; // the last position relaxed is j = n
        f[U] = m + cj;
        lq[U] = r.L + Q;
        r.L = Ln;
        r.cp1 = cn1;
        r.cp2 = cn2;
        r.t0 = r.t1;
        r.t1 = r.t2;
        r.t2 = t3;
        return true;
    }
};

template <int R, int F, int G, int E, bool CHK, int... Us>
__device__ __forceinline__ bool dp_block(int (&f)[R], int (&lq)[R], DpRegs &r, const uint8_t *row,
                                         CInt *tab, int j0, int n, int Q,
                                         std::integer_sequence<int, Us...>)
{
    return (DpState<R, F, G, E, Us, CHK>::run(f, lq, r, row, tab, j0, n, Q) && ...);
}

// Returns m_n of the lane's scenario; sets ovf when a window left the ring.
template <int R, int F, int G, int E>
__device__ __forceinline__ int dp_lane(const uint8_t *row, CInt *tab, int n, int f0, int Q,
                                       bool &ovf)
{
    int f[R], lq[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        f[i] = kInf;
        lq[i] = kNeg;
    }
    f[0] = f0; // p = 0: V(0) + a_1
    lq[0] = Q; // L_0 + Q
    DpRegs r;
    r.mres = kInf;
    r.ovf = 0;
    r.cp1 = ~0ull; // position 1 starts in the tail
    r.cp2 = ~0ull;
    r.t0 = tab_at(tab, 1);
    r.t1 = tab_at(tab, 2);
    r.t2 = tab_at(tab, 3);
    r.L = row[r.t0.x];
    r.qa = row[r.t1.x];
    int j0 = 0;
    for (; j0 + R - 1 <= n; j0 += R) // blocks whose positions all exist
        dp_block<R, F, G, E, false>(f, lq, r, row, tab, j0, n, Q,
                                    std::make_integer_sequence<int, R>{});
    if (j0 <= n) // the last, partial block
        dp_block<R, F, G, E, true>(f, lq, r, row, tab, j0, n, Q,
                                   std::make_integer_sequence<int, R>{});
    ovf = r.ovf != 0;
    return r.mres;
}


struct DpRegsO {
    int L;       // load of positions 1..j (at the start of position j)
    int2 t0;     // table entry of position j {customer, c}
    int2 t1;     // table entry of position j+1 (in flight)
    uint64_t cp1; // lanes rejecting d = F at position j (computed at j-1)
    uint64_t cp2; // lanes rejecting d = F + G at position j (computed at j-1)
    int mres;     // m of the last position relaxed (m_n after the loop)
    int ovf;      // 1 when a window reached past the ring
    // demand bytes of the lane's row, 32 positions per pair of registers:
    // a holds bytes [j0, j0 + 32) and b bytes [j0 + 32, j0 + 64) of the
    // current 64-position block; each is refilled with the bytes 64
    // further on once its last byte has been read
    u32x4 a[2], b[2];
};

__device__ __forceinline__ int byte_at(const u32x4 (&seg)[2], int b)
{
    const u32x4 &v = seg[b >> 4];
    const int w = (b >> 2) & 3;
    const uint32_t x = w == 0 ? v.x : w == 1 ? v.y : w == 2 ? v.z : v.w;
    return (int)((x >> (8 * (b & 3))) & 0xFFu);
}

// Position j = j0 + 1 + U of a 64-position block (j0 a multiple of 64).
// The two 32-byte halves a and b stay in fixed registers: a is refilled
// at U = 31, 32 positions before its next use, and b at U = 63, so no
// register ever copies a load in flight (a rotation cur <- nxt would, and
// would make the wave wait for the load at every block).
template <int R, int F, int G, int E, int U> struct DpStateO {
    __device__ __forceinline__ static void run(int (&f)[R], int (&lq)[R], DpRegsO &r,
                                               GU32x4 *row, int64_t segs, CInt *tab, int j0,
                                               int Q)
    {
        constexpr int SL = (U + 1) & (R - 1);
        constexpr int B = U & 31;
        const int j = j0 + 1 + U;
        // demand of position j + 1: byte U + 1 of the block
        const int qn = U == 31 ? byte_at(r.b, 0)
                       : U == 63 ? byte_at(r.a, 0)
                       : U < 32  ? byte_at(r.a, B + 1)
                                 : byte_at(r.b, B + 1);
        const int cj = r.t0.y;
        const int Ln = r.L + qn;
        r.t0 = r.t1;
        r.t1 = tab_at(tab, j + 2);
        uint64_t cn1, cn2;
        const int m = WindowMin<R, F, G, E>::template run<SL>(f, lq, r.L, Ln, j, r.cp1, r.cp2,
                                                              cn1, cn2, r.ovf);
        r.mres = m;
        f[SL] = m + cj;
        lq[SL] = r.L + Q;
        r.L = Ln;
        r.cp1 = cn1;
        r.cp2 = cn2;
        if (U == 31 || U == 63) {
            const int64_t seg = (j0 >> 5) + (U == 31 ? 2 : 3);
            u32x4(&dst)[2] = U == 31 ? r.a : r.b;
            if (seg < segs) {
                dst[0] = __builtin_nontemporal_load(row + 2 * seg);
                dst[1] = __builtin_nontemporal_load(row + 2 * seg + 1);
            }
        }
    }
};

template <int R, int F, int G, int E, int... Us>
__device__ __forceinline__ void dp_block_o(int (&f)[R], int (&lq)[R], DpRegsO &r, GU32x4 *row,
                                           int64_t segs, CInt *tab, int j0, int Q,
                                           std::integer_sequence<int, Us...>)
{
    (DpStateO<R, F, G, E, Us>::run(f, lq, r, row, segs, tab, j0, Q), ...);
}

// the tour's last block, positions j0 + 1 .. j0 + cnt (cnt < 64)
template <int R, int F, int G, int E, int... Us>
__device__ __forceinline__ void dp_partial_o(int (&f)[R], int (&lq)[R], DpRegsO &r, GU32x4 *row,
                                             int64_t segs, CInt *tab, int j0, int cnt, int Q,
                                             std::integer_sequence<int, Us...>)
{
    ((Us < cnt ? (DpStateO<R, F, G, E, Us>::run(f, lq, r, row, segs, tab, j0, Q), 0) : 0), ...);
}

template <int R, int F, int G, int E>
__device__ __forceinline__ int dp_lane_ordered(const uint8_t *rowb, int pitch, CInt *tab, int n,
                                               int f0, int Q, bool &ovf)
{
    int f[R], lq[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        f[i] = kInf;
        lq[i] = kNeg;
    }
    f[0] = f0;
    lq[0] = Q;
    DpRegsO r;
    r.mres = kInf;
    r.ovf = 0;
    r.cp1 = ~0ull; // position 1 starts in the tail
    r.cp2 = ~0ull;
    r.t0 = tab_at(tab, 1);
    r.t1 = tab_at(tab, 2);
    GU32x4 *row = (GU32x4 *)reinterpret_cast<const u32x4 *>(rowb);
    const int64_t segs = pitch / 32;
    r.a[0] = __builtin_nontemporal_load(row);
    r.a[1] = __builtin_nontemporal_load(row + 1);
    if (segs > 1) {
        r.b[0] = __builtin_nontemporal_load(row + 2);
        r.b[1] = __builtin_nontemporal_load(row + 3);
    } else {
        r.b[0] = u32x4{0u, 0u, 0u, 0u};
        r.b[1] = r.b[0];
    }
    r.L = byte_at(r.a, 0);
    int j0 = 0;
    for (; j0 + 64 <= n; j0 += 64) // blocks whose positions all exist
        dp_block_o<R, F, G, E>(f, lq, r, row, segs, tab, j0, Q,
                               std::make_integer_sequence<int, 64>{});
    if (j0 < n) // the last, partial block
        dp_partial_o<R, F, G, E>(f, lq, r, row, segs, tab, j0, n - j0, Q,
                                 std::make_integer_sequence<int, 64>{});
    ovf = r.ovf != 0;
    return r.mres;
}


// ---------------------------------------------------------------------------
// exact recursion for one lane straight from the definition (any window
// length, any demand value): V laid out [j][64] in global scratch, demands
// read through the tour from the lane's int16 row.  Returns V(n) (>= kInf
// when no split exists); negq reports a negative demand.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int exact_lane(const int16_t *__restrict__ qrow,
                                          const int2 *__restrict__ tab,
                                          const int2 *__restrict__ ab, int n, int Q, int *V,
                                          int lane, bool &negq)
{
    V[lane] = 0; // V(0)
    for (int j = 1; j <= n; ++j) {
        const int bj = ab[j - 1].y;
        int best = kInf;
        int load = 0;
        for (int p = j - 1; p >= 0; --p) {
            const int q = qrow[tab[p + 1].x];
            negq = negq || q < 0;
            load += q;
            if (load > Q)
                break;
            const int vp = V[(int64_t)p * kWave + lane];
            if (vp < kInf)
                best = min(best, vp + ab[p].x + bj);
        }
        V[(int64_t)j * kWave + lane] = best;
    }
    return V[(int64_t)n * kWave + lane];
}

} // namespace splitk
