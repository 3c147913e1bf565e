"""Generates window_min_multi_asm.inc: the masked window minimum of one tour
position over L potential rings that share one admissibility window (the
passes of a fleet-bounded split: every pass relaxes the same predecessor
window, with its own potentials).  Run after editing:
    python gen_multiring_asm.py

The block is the one of gen_window_asm.py with every `v_min` repeated once
per ring: the lane masks, the head checks, the exec narrowing and the exits
are computed once for all rings.  Operand d-1 of ring l is f<l>_<d>, the
potential of predecessor p = j - d in ring l; q<d> its threshold.
Outputs m<l> (2^30 if no admissible predecessor), cn1, cn2, ov as in
window_min_asm.inc.
Variants (R, F, G, E, L) are named M<F>_<G>_<E>_L<L>.
"""
import os

from gen_window_asm import exits

HERE = os.path.dirname(os.path.abspath(__file__))
INF_IMM = "2.0"
# (ring, first, group, every) of the hard-capacity fleet passes, and ring counts
VARIANTS = ((32, 8, 3, 3), (64, 16, 4, 4))
RING_COUNTS = (2, 3)


def block(R, first, group, every, L):
    out = []
    a = out.append
    head_end = first + group
    xs = exits(R, head_end, every)

    def cell(d):
        a("v_cmpx_le_i32_e32 vcc, %%[L], %%[q%d]" % d)
        if d in xs:
            a("s_cbranch_execz .Ldone_%=")
        for l in range(L):
            a("v_min_i32_e32 %%[m%d], %%[m%d], %%[f%d_%d]" % (l, l, l, d))

    def fold(lo, hi, start):
        cells = list(range(lo, hi + 1))
        for l in range(L):
            k = 0
            if start:
                a("v_min_i32_e32 %%[m%d], %%[f%d_%d], %%[f%d_%d]" % (l, l, cells[0], l, cells[1]))
                k = 2
            while k < len(cells):
                if k + 1 < len(cells):
                    a("v_min3_i32 %%[m%d], %%[m%d], %%[f%d_%d], %%[f%d_%d]" % (l, l, l, cells[k], l, cells[k + 1]))
                    k += 2
                else:
                    a("v_min_i32_e32 %%[m%d], %%[m%d], %%[f%d_%d]" % (l, l, l, cells[k]))
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
    a(".Lt%d_%%=:" % (head_end + 1))
    for d in range(head_end + 1, R + 1):
        cell(d)
    a("s_cmp_gt_i32 %%[j], %d" % R)
    a("s_cbranch_scc0 .Ldone_%=")
    a("v_mov_b32_e32 %[ov], 1")
    a("s_branch .Ldone_%=")
    if group:
        a(".Lt%d_%%=:" % (first + 1))
        for d in range(first + 1, head_end + 1):
            cell(d)
        a("s_branch .Lt%d_%%=" % (head_end + 1))
    a(".Lt1_%=:")
    for l in range(L):
        a("v_mov_b32_e32 %%[m%d], %s" % (l, INF_IMM))
    for d in range(1, first + 1):
        cell(d)
    a("s_branch .Lt%d_%%=" % (first + 1))
    a(".Ldone_%=:")
    a("s_mov_b64 exec, %[sv]")
    return out


def name(R, first, group, every, L):
    return "R%d_M%d_%d_%d_L%d" % (R, first, group, every, L)


def emit(R, first, group, every, L):
    out = ["#define SPLIT_MULTI_ASM_%s \\" % name(R, first, group, every, L)]
    for ins in block(R, first, group, every, L):
        out.append('    "%s\\n" \\' % ins)
    out.append('    ""')
    out.append("")
    return "\n".join(out)


def emit_wrapper(R, first, group, every, L):
    ms = ", ".join('[m%d] "=&v"(m[%d])' % (l, l) for l in range(L))
    fops = []
    for l in range(L):
        for d in range(1, R + 1):
            fops.append('[f%d_%d] "v"(f[%d][((U) - %d) & %d])' % (l, d, l, d, R - 1))
    qops = ['[q%d] "v"(lq[((U) - %d) & %d])' % (d, d, R - 1) for d in range(1, R + 1)]
    lines = [
        "template <> struct WindowMinMulti<%d, %d, %d, %d, %d> {" % (R, first, group, every, L),
        "    template <int U>",
        "    __device__ __forceinline__ static void run(const int (&f)[%d][%d], const int (&lq)[%d]," % (L, R, R),
        "                                               int L, int Ln, int j, uint64_t cp1, uint64_t cp2,",
        "                                               uint64_t &cn1, uint64_t &cn2, int &ov, int (&m)[%d])" % L,
        "    {",
        "        uint64_t sv;",
        "        asm volatile(SPLIT_MULTI_ASM_%s" % name(R, first, group, every, L),
        "                     : %s, [ov] \"+v\"(ov), [sv] \"=&s\"(sv), [cn1] \"=&s\"(cn1)%s" % (
            ms, ', [cn2] "=&s"(cn2)' if group else ""),
        "                     : [L] \"v\"(L), [Ln] \"v\"(Ln), [j] \"s\"(j), [cp1] \"s\"(cp1)%s," % (
            ', [cp2] "s"(cp2)' if group else ""),
        "                       " + ",\n                       ".join(fops + qops),
        '                     : "vcc", "scc");',
    ]
    if not group:
        lines.append("        (void)cp2;")
        lines.append("        cn2 = 0;")
    lines += ["    }", "};", ""]
    return "\n".join(lines)


def render() -> str:
    """The generated file's text."""
    text = ["// window_min_multi_asm.inc -- GENERATED by gen_multiring_asm.py; do not edit.",
            "// Masked window minimum of one tour position over L rings sharing one window",
            "// (see gen_multiring_asm.py).",
            "// WindowMinMulti<R, F, G, E, L>::run<U>(f, lq, L, Ln, j, cp1, cp2, cn1, cn2, ov, m).",
            "",
            "template <int R, int F, int G, int E, int L> struct WindowMinMulti;",
            ""]
    for R, first, group, every in VARIANTS:
        for L in RING_COUNTS:
            text.append(emit(R, first, group, every, L))
            text.append(emit_wrapper(R, first, group, every, L))
    return "\n".join(text)


def main():
    path = os.path.join(HERE, "window_min_multi_asm.inc")
    with open(path, "w") as fh:
        fh.write(render())
    print(path)


if __name__ == "__main__":
    main()
