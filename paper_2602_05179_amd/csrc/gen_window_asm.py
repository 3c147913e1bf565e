"""Generates window_min_asm.inc: the masked window minimum of one tour
position as gfx950 inline-assembly blocks.  Run after editing:
    python gen_window_asm.py

Operand d-1 of a block always holds predecessor p = j - d (the caller
passes the ring slots rotated), so one text serves every unrolled position.

Inputs : L (load of positions 1..j), j (uniform), f_d, lq_d for d = 1..R
         (potential V(p) + a_{p+1} and threshold L_p + Q of p = j - d).
Outputs: m = min over admissible d of f_d (2^30 if none),
         ov = 1 on lanes that admit d = R while j > R (window past the ring).

Admissible predecessors of a lane form the contiguous range d = 1..w, so a
lane that rejects d rejects every larger d.  A block has two regimes:

  head : cells every active lane admits.  A group of cells is validated by
         one v_cmp on its farthest cell (all lanes admit it => all admit the
         group) and folded with v_min3, two potentials per instruction.
         The first group spans `first` cells (checked once), later groups
         are pairs.  The first group that fails sends control to the tail
         entry at the group's first cell.
  tail : v_cmpx narrows EXEC to the lanes still admitting d, then v_min.
         Every `every` cells a branch leaves once EXEC is empty (cells
         executed after EXEC emptied are no-ops).  EXEC is restored once.

Variants (first, every) are named V<first>_<every>.
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
INF_IMM = "2.0"  # inline constant with bit pattern 0x40000000 = 2^30
# (first, every) schedules compiled for each ring length
VARIANTS = {
    32: ((0, 1), (8, 2), (8, 3), (6, 3), (4, 3), (8, 4)),
    64: ((0, 1), (8, 3), (16, 3), (24, 3)),
}
RINGS = tuple(VARIANTS)


def head_groups(R, first):
    """[(lo, hi)] cell ranges of the head groups, in order."""
    groups = []
    d = 1
    if first:
        groups.append((1, first))
        d = first + 1
    while d + 1 <= R:
        groups.append((d, d + 1))
        d += 2
    return groups


def block(R: int, first: int, every: int) -> list:
    L = []
    a = L.append
    a("s_mov_b64 %[sv], exec")
    groups = head_groups(R, first)
    for gi, (lo, hi) in enumerate(groups):
        a("v_cmp_le_i32_e64 %%[c], %%[L], %%[q%d]" % hi)
        a("s_cmp_eq_u64 %[c], exec")
        a("s_cbranch_scc0 .Lt%d_%%=" % lo)
        cells = list(range(lo, hi + 1))
        k = 0
        if gi == 0:
            if len(cells) == 1:
                a("v_mov_b32_e32 %%[m], %%[f%d]" % cells[0])
                k = 1
            else:
                a("v_min_i32_e32 %%[m], %%[f%d], %%[f%d]" % (cells[0], cells[1]))
                k = 2
        while k < len(cells):
            if k + 1 < len(cells):
                a("v_min3_i32 %%[m], %%[m], %%[f%d], %%[f%d]" % (cells[k], cells[k + 1]))
                k += 2
            else:
                a("v_min_i32_e32 %%[m], %%[m], %%[f%d]" % cells[k])
                k += 1
    # every lane admits all R slots
    a("s_cmp_gt_i32 %%[j], %d" % R)
    a("s_cbranch_scc0 .Ldone_%=")
    a("v_mov_b32_e32 %[ov], 1")
    a("s_branch .Ldone_%=")
    # tail cells
    entries = {lo for lo, _ in groups}
    a(".Lt1_%=:")
    a("v_mov_b32_e32 %%[m], %s" % INF_IMM)
    since = 0
    for d in range(1, R + 1):
        if d in entries and d > 1:
            a(".Lt%d_%%=:" % d)
            since = 0
        a("v_cmpx_le_i32_e32 vcc, %%[L], %%[q%d]" % d)
        since += 1
        nxt_entry = (d + 1) in entries
        if since >= every or nxt_entry or d == R:
            a("s_cbranch_execz .Ldone_%=")
            since = 0
        a("v_min_i32_e32 %%[m], %%[m], %%[f%d]" % d)
    # lanes left admit d = R
    a("s_cmp_gt_i32 %%[j], %d" % R)
    a("s_cbranch_scc0 .Ldone_%=")
    a("v_mov_b32_e32 %[ov], 1")
    a(".Ldone_%=:")
    a("s_mov_b64 exec, %[sv]")
    return L


def emit(R: int, first: int, every: int) -> str:
    out = ["#define SPLIT_WINDOW_ASM_R%d_V%d_%d \\" % (R, first, every)]
    for ins in block(R, first, every):
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


def emit_wrapper(R: int, first: int, every: int) -> str:
    return "\n".join([
        "template <> struct WindowMin<%d, %d, %d> {" % (R, first, every),
        "    template <int U>",
        "    __device__ __forceinline__ static int run(const int (&f)[%d], const int (&lq)[%d], int L," % (R, R),
        "                                              int j, int &ov)",
        "    {",
        "        int m;",
        "        uint64_t sv, c;",
        "        asm volatile(SPLIT_WINDOW_ASM_R%d_V%d_%d" % (R, first, every),
        "                     : [m] \"=&v\"(m), [ov] \"+v\"(ov), [sv] \"=&s\"(sv), [c] \"=&s\"(c)",
        "                     : [L] \"v\"(L), [j] \"s\"(j), SPLIT_WINDOW_OPERANDS_R%d(f, lq, U)" % R,
        "                     : \"vcc\", \"scc\");",
        "        return m;",
        "    }",
        "};",
        ""])


def main():
    text = ["// window_min_asm.inc -- GENERATED by gen_window_asm.py; do not edit.",
            "// Masked window minimum of one tour position (see gen_window_asm.py).",
            "// WindowMin<R, FIRST, EVERY>::run<U>(f, lq, L, j, ov) returns m.",
            "",
            "template <int R, int FIRST, int EVERY> struct WindowMin;",
            ""]
    for R in RINGS:
        text.append(emit_operands(R))
        for first, every in VARIANTS[R]:
            text.append(emit(R, first, every))
            text.append(emit_wrapper(R, first, every))
    text.append("#define SPLIT_WINDOW_VARIANTS(X) \\")
    combos = [(R, f, e) for R in RINGS for f, e in VARIANTS[R]]
    for k, (R, f, e) in enumerate(combos):
        text.append("    X(%d, %d, %d)%s" % (R, f, e, " \\" if k + 1 < len(combos) else ""))
    text.append("")
    path = os.path.join(HERE, "window_min_asm.inc")
    with open(path, "w") as f:
        f.write("\n".join(text))
    print(path)


if __name__ == "__main__":
    main()
