"""Generates window_min_asm.inc: the masked window minimum of one tour
position as gfx950 inline-assembly blocks.  Run after editing:
    python gen_window_asm.py

Operand d-1 of a block always holds predecessor p = j - d (the caller
passes the ring slots rotated), so one text serves every unrolled position.

Inputs : L (load of positions 1..j), Ln (load of positions 1..j+1),
         j (uniform), f_d, lq_d for d = 1..R (potential V(p) + a_{p+1} and
         threshold L_p + Q of p = j - d), cp1 / cp2 (lanes that reject
         d = F / d = F + G at this position, computed by the previous
         position's block).
Outputs: m  = min over admissible d of f_d (2^30 if none),
         cn1 / cn2 = the same two masks for position j + 1 (Ln against the
              thresholds of p = j + 1 - F and p = j + 1 - F - G, which are
              this block's operands F - 1 and F + G - 1),
         ov = 1 on lanes that admit d = R while j > R (window past the ring).

Admissible predecessors of a lane form the contiguous range d = 1..w, so a
lane that rejects d rejects every larger d.  A block has two regimes:

  head : cells every active lane admits, folded with v_min3 (two potentials
         per instruction): cells 1..F, then (G > 0) cells F+1..F+G.  Each
         group is validated by a mask computed one position earlier, so its
         branch is a scalar test that never waits on a vector compare.  A
         failing group sends control to the tail entry at its first cell.
  tail : v_cmpx narrows EXEC to the lanes still admitting d, then v_min.
         Every E cells a branch leaves once EXEC is empty (cells executed
         after EXEC emptied are no-ops).  EXEC is restored once.

The path where every group passes falls straight into the tail; the other
tail entries are laid out after it and jump back in.
Variants (F, G, E) are named V<F>_<G>_<E>.
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
INF_IMM = "2.0"  # inline constant with bit pattern 0x40000000 = 2^30
# (first, group, every) schedules compiled for each ring length
VARIANTS = {
    32: ((8, 3, 3), (8, 0, 4), (8, 3, 2), (8, 2, 2), (6, 3, 3), (6, 2, 2), (10, 3, 3)),
    64: ((16, 4, 4), (16, 0, 6), (20, 4, 3), (12, 6, 2), (24, 4, 4)),
}
RINGS = tuple(VARIANTS)


def exits(R, head_end, every):
    """Tail cells after which an empty EXEC leaves the block."""
    xs = set(range(every, head_end, every))
    xs.update(range(head_end + every, R + 1, every))
    xs.add(R)
    return xs


def block(R: int, first: int, group: int, every: int) -> list:
    assert 2 <= first and first + group < R and group >= 0 and every >= 1
    assert group != 1
    L = []
    a = L.append
    head_end = first + group
    xs = exits(R, head_end, every)

    def cell(d):
        a("v_cmpx_le_i32_e32 vcc, %%[L], %%[q%d]" % d)
        if d in xs:
            a("s_cbranch_execz .Ldone_%=")
        a("v_min_i32_e32 %%[m], %%[m], %%[f%d]" % d)

    def fold(lo, hi, start):
        cells = list(range(lo, hi + 1))
        k = 0
        if start:
            a("v_min_i32_e32 %%[m], %%[f%d], %%[f%d]" % (cells[0], cells[1]))
            k = 2
        while k < len(cells):
            if k + 1 < len(cells):
                a("v_min3_i32 %%[m], %%[m], %%[f%d], %%[f%d]" % (cells[k], cells[k + 1]))
                k += 2
            else:
                a("v_min_i32_e32 %%[m], %%[m], %%[f%d]" % cells[k])
                k += 1

    a("s_mov_b64 %[sv], exec")
    a("v_cmp_gt_i32_e64 %%[cn1], %%[Ln], %%[q%d]" % (first - 1))
    if group:
        a("v_cmp_gt_i32_e64 %%[cn2], %%[Ln], %%[q%d]" % (head_end - 1))
    a("s_cmp_lg_u64 %[cp1], 0")
    a("s_cbranch_scc1 .Lt1_%=")
    fold(1, first, True)
    if group:
        a("s_cmp_lg_u64 %[cp2], 0")
        a("s_cbranch_scc1 .Lt%d_%%=" % (first + 1))
        fold(first + 1, head_end, False)
    # hot tail: every head group passed, cells head_end+1..R
    a(".Lt%d_%%=:" % (head_end + 1))
    for d in range(head_end + 1, R + 1):
        cell(d)
    # lanes left admit d = R
    a("s_cmp_gt_i32 %%[j], %d" % R)
    a("s_cbranch_scc0 .Ldone_%=")
    a("v_mov_b32_e32 %[ov], 1")
    a("s_branch .Ldone_%=")
    if group:
        # the second group failed: its cells, then back into the hot tail
        a(".Lt%d_%%=:" % (first + 1))
        for d in range(first + 1, head_end + 1):
            cell(d)
        a("s_branch .Lt%d_%%=" % (head_end + 1))
    # the first group failed: cells 1..F, then on as above
    a(".Lt1_%=:")
    a("v_mov_b32_e32 %%[m], %s" % INF_IMM)
    for d in range(1, first + 1):
        cell(d)
    a("s_branch .Lt%d_%%=" % (first + 1))
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
    if group:
        outs = ('                     : [m] "=&v"(m), [ov] "+v"(ov), [sv] "=&s"(sv), [cn1] "=&s"(cn1),\n'
                '                       [cn2] "=&s"(cn2)')
        ins = '                     : [L] "v"(L), [Ln] "v"(Ln), [j] "s"(j), [cp1] "s"(cp1), [cp2] "s"(cp2),'
        tail = ""
    else:
        outs = '                     : [m] "=&v"(m), [ov] "+v"(ov), [sv] "=&s"(sv), [cn1] "=&s"(cn1)'
        ins = '                     : [L] "v"(L), [Ln] "v"(Ln), [j] "s"(j), [cp1] "s"(cp1),'
        tail = "        (void)cp2;\n        cn2 = 0;\n"
    return "\n".join([
        "template <> struct WindowMin<%d, %d, %d, %d> {" % (R, first, group, every),
        "    template <int U>",
        "    __device__ __forceinline__ static int run(const int (&f)[%d], const int (&lq)[%d], int L," % (R, R),
        "                                              int Ln, int j, uint64_t cp1, uint64_t cp2,",
        "                                              uint64_t &cn1, uint64_t &cn2, int &ov)",
        "    {",
        "        int m;",
        "        uint64_t sv;",
        "        asm volatile(SPLIT_WINDOW_ASM_R%d_%s" % (R, name(first, group, every)),
        outs,
        ins,
        "                       SPLIT_WINDOW_OPERANDS_R%d(f, lq, U)" % R,
        '                     : "vcc", "scc");',
        tail + "        return m;",
        "    }",
        "};",
        ""])


def render() -> str:
    """The generated file's text."""
    text = ["// window_min_asm.inc -- GENERATED by gen_window_asm.py; do not edit.",
            "// Masked window minimum of one tour position (see gen_window_asm.py).",
            "// WindowMin<R, F, G, E>::run<U>(f, lq, L, Ln, j, cp1, cp2, cn1, cn2, ov) returns m.",
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
    return "\n".join(text)


def main():
    path = os.path.join(HERE, "window_min_asm.inc")
    with open(path, "w") as fh:
        fh.write(render())
    print(path)


if __name__ == "__main__":
    main()
