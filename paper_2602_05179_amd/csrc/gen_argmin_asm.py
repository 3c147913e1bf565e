"""Generates window_argmin_asm.inc: the masked window minimum of one tour
position together with its smallest minimising predecessor, as gfx950
inline-assembly blocks (the route-recovery recursion).  Run after editing:
    python gen_argmin_asm.py

Operand d-1 of a block holds predecessor p = j - d (the caller passes the
ring slots rotated), as in window_min_asm.inc.

Inputs : L (load of positions 1..j), Ln (load of positions 1..j+1),
         j (uniform), f_d, lq_d for d = 1..R, cp1 (lanes that reject d = F
         at this position, computed by the previous position's block).
Outputs: m  = min over admissible d of f_d (2^30 if none),
         a  = the LARGEST admissible d with f_d = m (0 if none), i.e. the
              smallest minimising predecessor p = j - a,
         cn1 = lanes that reject d = F at position j + 1,
         ov = 1 on lanes that admit d = R while j > R (window past the ring).

Cells are visited in increasing d.  A cell updates the running minimum and
then compares it with its own potential: equality means f_d is at most
every earlier potential, so the cell becomes the argmin; ties therefore go
to the larger d (the smaller p).

  head : (F > 0) when no active lane rejects d = F, cells 1..F are folded
         with v_min3 and then compared with the head minimum in increasing
         d, without per-cell masking;
  tail : v_cmpx narrows EXEC to the lanes still admitting d, then min,
         compare, select.  Every E cells a branch leaves once EXEC is empty.
Variants (F, E) are named A<F>_<E>.
"""
import os

from gen_window_asm import exits

HERE = os.path.dirname(os.path.abspath(__file__))
INF_IMM = "2.0"  # inline constant with bit pattern 0x40000000 = 2^30
# (first, every) schedules compiled for each ring length
VARIANTS = {
    32: ((6, 3),),
    64: ((12, 4),),
}
RINGS = tuple(VARIANTS)


def block(R: int, first: int, every: int) -> list:
    assert first == 0 or 2 <= first < R
    assert every >= 1
    L = []
    a = L.append
    xs = exits(R, first, every)

    def cell(d):
        a("v_cmpx_le_i32_e32 vcc, %%[L], %%[q%d]" % d)
        if d in xs:
            a("s_cbranch_execz .Ldone_%=")
        a("v_min_i32_e32 %%[m], %%[m], %%[f%d]" % d)
        select(d)

    def select(d):
        # vcc = (m != f_d): keep a; else a = d
        a("v_cmp_ne_u32_e32 vcc, %%[m], %%[f%d]" % d)
        a("v_cndmask_b32_e32 %%[a], %d, %%[a], vcc" % d)

    a("s_mov_b64 %[sv], exec")
    a("v_mov_b32_e32 %[a], 0")
    if first:
        a("v_cmp_gt_i32_e64 %%[cn1], %%[Ln], %%[q%d]" % (first - 1))
        a("s_cmp_lg_u64 %[cp1], 0")
        a("s_cbranch_scc1 .Lt1_%=")
        cells = list(range(1, first + 1))
        a("v_min_i32_e32 %%[m], %%[f%d], %%[f%d]" % (cells[0], cells[1]))
        k = 2
        while k < len(cells):
            if k + 1 < len(cells):
                a("v_min3_i32 %%[m], %%[m], %%[f%d], %%[f%d]" % (cells[k], cells[k + 1]))
                k += 2
            else:
                a("v_min_i32_e32 %%[m], %%[m], %%[f%d]" % cells[k])
                k += 1
        for d in cells:
            select(d)
        a(".Lt%d_%%=:" % (first + 1))
    else:
        a("v_mov_b32_e32 %%[m], %s" % INF_IMM)
    for d in range(first + 1, R + 1):
        cell(d)
    a("s_cmp_gt_i32 %%[j], %d" % R)
    a("s_cbranch_scc0 .Ldone_%=")
    a("v_mov_b32_e32 %[ov], 1")
    if first:
        a("s_branch .Ldone_%=")
        # the head check failed: cells 1..F masked, then back into the tail
        a(".Lt1_%=:")
        a("v_mov_b32_e32 %%[m], %s" % INF_IMM)
        for d in range(1, first + 1):
            cell(d)
        a("s_branch .Lt%d_%%=" % (first + 1))
    a(".Ldone_%=:")
    a("s_mov_b64 exec, %[sv]")
    return L


def name(first, every):
    return "A%d_%d" % (first, every)


def emit(R: int, first: int, every: int) -> str:
    out = ["#define SPLIT_ARGMIN_ASM_R%d_%s \\" % (R, name(first, every))]
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
    out = ["#define SPLIT_ARGMIN_OPERANDS_R%d(F, LQ, U) \\" % R]
    for k, o in enumerate(ops):
        out.append("    " + o + (", \\" if k + 1 < len(ops) else ""))
    out.append("")
    return "\n".join(out)


def emit_wrapper(R: int, first: int, every: int) -> str:
    if first:
        outs = ('                     : [m] "=&v"(m), [a] "=&v"(a), [ov] "+v"(ov), [sv] "=&s"(sv),\n'
                '                       [cn1] "=&s"(cn1)')
        ins = '                     : [L] "v"(L), [Ln] "v"(Ln), [j] "s"(j), [cp1] "s"(cp1),'
        tail = ""
    else:
        outs = '                     : [m] "=&v"(m), [a] "=&v"(a), [ov] "+v"(ov), [sv] "=&s"(sv)'
        ins = '                     : [L] "v"(L), [j] "s"(j),'
        tail = "        (void)Ln;\n        (void)cp1;\n        cn1 = 0;\n"
    return "\n".join([
        "template <> struct WindowArgmin<%d, %d, %d> {" % (R, first, every),
        "    template <int U>",
        "    __device__ __forceinline__ static int run(const int (&f)[%d], const int (&lq)[%d], int L," % (R, R),
        "                                              int Ln, int j, uint64_t cp1, uint64_t &cn1,",
        "                                              int &a, int &ov)",
        "    {",
        "        int m;",
        "        uint64_t sv;",
        "        asm volatile(SPLIT_ARGMIN_ASM_R%d_%s" % (R, name(first, every)),
        outs,
        ins,
        "                       SPLIT_ARGMIN_OPERANDS_R%d(f, lq, U)" % R,
        '                     : "vcc", "scc");',
        tail + "        return m;",
        "    }",
        "};",
        ""])


def render() -> str:
    """The generated file's text."""
    text = ["// window_argmin_asm.inc -- GENERATED by gen_argmin_asm.py; do not edit.",
            "// Masked window minimum and smallest minimising predecessor of one tour",
            "// position (see gen_argmin_asm.py).",
            "// WindowArgmin<R, F, E>::run<U>(f, lq, L, Ln, j, cp1, cn1, a, ov) returns m.",
            "",
            "template <int R, int F, int E> struct WindowArgmin;",
            ""]
    for R in RINGS:
        text.append(emit_operands(R))
        for first, every in VARIANTS[R]:
            text.append(emit(R, first, every))
            text.append(emit_wrapper(R, first, every))
    text.append("#define SPLIT_ARGMIN_VARIANTS(X) \\")
    combos = [(R, f, e) for R in RINGS for f, e in VARIANTS[R]]
    for k, (R, f, e) in enumerate(combos):
        text.append("    X(%d, %d, %d)%s" % (R, f, e, " \\" if k + 1 < len(combos) else ""))
    text.append("")
    return "\n".join(text)


def main():
    path = os.path.join(HERE, "window_argmin_asm.inc")
    with open(path, "w") as fh:
        fh.write(render())
    print(path)


if __name__ == "__main__":
    main()
