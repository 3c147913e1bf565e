"""Generates window_min_asm.inc: the masked window minimum of one tour
position as gfx950 inline-assembly blocks.  Run after editing:
    python gen_window_asm.py

Operand d-1 of a block always holds predecessor p = j - d (the caller
passes the ring slots rotated), so one text serves every unrolled position.

Inputs : L (load of positions 1..j), Ln (load of positions 1..j+1),
         j (uniform), f_d, lq_d for d = 1..R (potential V(p) + a_{p+1} and
         threshold L_p + Q of p = j - d), cp (lanes that reject d = F at
         this position, computed by the previous position's block).
Outputs: m  = min over admissible d of f_d (2^30 if none),
         cn = lanes that will reject d = F at position j + 1
              (Ln > lq of p = j + 1 - F, i.e. this block's operand F - 1),
         ov = 1 on lanes that admit d = R while j > R (window past the ring).

Admissible predecessors of a lane form the contiguous range d = 1..w, so a
lane that rejects d rejects every larger d.  A block has two regimes:

  head : cells every active lane admits, folded with v_min3 (two potentials
         per instruction).  The first group, cells 1..F, is validated by a
         mask computed one position earlier, so its branch never waits on a
         fresh vector compare.  Later groups of G cells (G = 0: none) are
         validated on their farthest cell by v_cmp into VCC and a branch on
         VCC.  A failing group sends control to the tail entry at the
         group's first cell.
  tail : v_cmpx narrows EXEC to the lanes still admitting d, then v_min.
         Every E cells a branch leaves once EXEC is empty (cells executed
         after EXEC emptied are no-ops).  EXEC is restored once.

Variants (F, G, E) are named V<F>_<G>_<E>.
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
INF_IMM = "2.0"  # inline constant with bit pattern 0x40000000 = 2^30
# (first, group, every) schedules compiled for each ring length
VARIANTS = {
    32: ((8, 0, 4), (8, 0, 3), (8, 0, 6), (6, 0, 4), (10, 0, 4), (8, 4, 4), (8, 2, 3)),
    64: ((16, 0, 6), (16, 0, 4), (24, 0, 4), (16, 4, 4), (8, 4, 4)),
}
RINGS = tuple(VARIANTS)


def head_groups(R, first, group):
    """[(lo, hi)] cell ranges of the head groups, in order."""
    groups = [(1, first)]
    d = first + 1
    while group and d + group - 1 <= R:
        groups.append((d, d + group - 1))
        d += group
    return groups


def exits(R, first, every):
    """Tail cells after which an empty EXEC leaves the block."""
    xs = set(range(every, first, every))
    xs.update(range(first + every, R + 1, every))
    xs.add(R)
    return xs


def block(R: int, first: int, group: int, every: int) -> list:
    assert 2 <= first < R and group >= 0 and every >= 1
    L = []
    a = L.append
    a("s_mov_b64 %[sv], exec")
    a("v_cmp_gt_i32_e64 %%[cn], %%[Ln], %%[q%d]" % (first - 1))
    a("s_cmp_lg_u64 %[cp], 0")
    a("s_cbranch_scc1 .Lt1_%=")
    groups = head_groups(R, first, group)
    for gi, (lo, hi) in enumerate(groups):
        cells = list(range(lo, hi + 1))
        k = 0
        if gi == 0:
            a("v_min_i32_e32 %%[m], %%[f%d], %%[f%d]" % (cells[0], cells[1]))
            k = 2
        else:
            a("v_cmp_gt_i32_e32 vcc, %%[L], %%[q%d]" % hi)
            a("s_cbranch_vccnz .Lt%d_%%=" % lo)
        while k < len(cells):
            if k + 1 < len(cells):
                a("v_min3_i32 %%[m], %%[m], %%[f%d], %%[f%d]" % (cells[k], cells[k + 1]))
                k += 2
            else:
                a("v_min_i32_e32 %%[m], %%[m], %%[f%d]" % cells[k])
                k += 1
    head_end = groups[-1][1]
    xs = exits(R, first, every)

    def cell(d):
        a("v_cmpx_le_i32_e32 vcc, %%[L], %%[q%d]" % d)
        if d in xs:
            a("s_cbranch_execz .Ldone_%=")
        a("v_min_i32_e32 %%[m], %%[m], %%[f%d]" % d)

    # hot tail: falls through from the head, cells head_end+1..R
    a(".Lt%d_%%=:" % (head_end + 1))
    for d in range(head_end + 1, R + 1):
        cell(d)
    # lanes left admit d = R
    a("s_cmp_gt_i32 %%[j], %d" % R)
    a("s_cbranch_scc0 .Ldone_%=")
    a("v_mov_b32_e32 %[ov], 1")
    a("s_branch .Ldone_%=")
    # cold tail: entered when a head group fails, cells 1..head_end, then
    # back into the hot tail
    entries = {lo for lo, _ in groups}
    a(".Lt1_%=:")
    a("v_mov_b32_e32 %%[m], %s" % INF_IMM)
    for d in range(1, head_end + 1):
        if d in entries and d > 1:
            a(".Lt%d_%%=:" % d)
        cell(d)
    a("s_branch .Lt%d_%%=" % (head_end + 1))
    a(".Ldone_%=:")
    a("s_mov_b64 exec, %[sv]")
    return L


def name(first, group, every):
    return "V%d_%d_%d" % (first, group, every)


def emit(R: int, first: int, group: int, every: int) -> str:
    out = ["#define SPLIT_WINDOW_ASM_R%d_%s \\" % (R, name(first, group, every))]
    for ins in block(R, first, group, every):
        out.append('    "%s\\n" \\' % ins)
    out.append('    ""')
    out.append("")
    return "\n".join(out)


def emit_operands(R: int) -> str:
    ops = []
    for d in range(1, R + 1):
        ops.append('[f%d] "v"(F[((U) - %d) & %d])' % (d, d, R - 1))
        ops.append('[q%d] "v"(LQ[((U) - %d) & %d])' % (d, d, R - 1))
    out = ["#define SPLIT_WINDOW_OPERANDS_R%d(F, LQ, U) \\" % R]
    for k, o in enumerate(ops):
        out.append("    " + o + (", \\" if k + 1 < len(ops) else ""))
    out.append("")
    return "\n".join(out)


def emit_wrapper(R: int, first: int, group: int, every: int) -> str:
    return "\n".join([
        "template <> struct WindowMin<%d, %d, %d, %d> {" % (R, first, group, every),
        "    template <int U>",
        "    __device__ __forceinline__ static int run(const int (&f)[%d], const int (&lq)[%d], int L," % (R, R),
        "                                              int Ln, int j, uint64_t cp, uint64_t &cn,",
        "                                              int &ov)",
        "    {",
        "        int m;",
        "        uint64_t sv;",
        "        asm volatile(SPLIT_WINDOW_ASM_R%d_%s" % (R, name(first, group, every)),
        "                     : [m] \"=&v\"(m), [ov] \"+v\"(ov), [sv] \"=&s\"(sv), [cn] \"=&s\"(cn)",
        "                     : [L] \"v\"(L), [Ln] \"v\"(Ln), [j] \"s\"(j), [cp] \"s\"(cp),",
        "                       SPLIT_WINDOW_OPERANDS_R%d(f, lq, U)" % R,
        "                     : \"vcc\", \"scc\");",
        "        return m;",
        "    }",
        "};",
        ""])


def main():
    text = ["// window_min_asm.inc -- GENERATED by gen_window_asm.py; do not edit.",
            "// Masked window minimum of one tour position (see gen_window_asm.py).",
            "// WindowMin<R, F, G, E>::run<U>(f, lq, L, Ln, j, cp, cn, ov) returns m.",
            "",
            "template <int R, int F, int G, int E> struct WindowMin;",
            ""]
    for R in RINGS:
        text.append(emit_operands(R))
        for first, group, every in VARIANTS[R]:
            text.append(emit(R, first, group, every))
            text.append(emit_wrapper(R, first, group, every))
    text.append("#define SPLIT_WINDOW_VARIANTS(X) \\")
    combos = [(R, f, g, e) for R in RINGS for f, g, e in VARIANTS[R]]
    for k, (R, f, g, e) in enumerate(combos):
        text.append("    X(%d, %d, %d, %d)%s" % (R, f, g, e, " \\" if k + 1 < len(combos) else ""))
    text.append("")
    path = os.path.join(HERE, "window_min_asm.inc")
    with open(path, "w") as f:
        f.write("\n".join(text))
    print(path)


if __name__ == "__main__":
    main()
