"""Writes the batched-kernel instantiation units zk_batch_{row,col}_{f64,f32}.hip
(one function per unit mapping a team shape (T, E, padded) to its kernel).  Run
from any directory; the units are committed, this script regenerates them."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# power-of-two axes: padded iff E % 3 == 0
POW2 = ([(T, E) for T in (2, 4, 8, 16) for E in (2, 3, 4, 6)]
        + [(T, E) for T in (32, 64, 128, 256) for E in (2, 3, 4, 6, 8, 12)]
        + [(512, E) for E in (2, 3, 4, 6)] + [(1024, E) for E in (2, 3)])
SHAPES = [(T, E, E % 3 == 0) for T, E in POW2]
# axes of n = 3 2^k points: padded transforms with E = 9, base transforms with E = 6
SHAPES += ([(T, 9, True) for T in (2, 4, 8, 16, 32, 64, 128, 256)]
           + [(T, 6, False) for T in (2, 4, 8, 16, 32, 64, 128, 256)])
# axes of n = 5 2^k points: padded transforms with E = 15, base transforms with E = 10
SHAPES += [(T, 15, True) for T in (2, 4, 8, 16, 32, 64, 128)] + [(T, 10, False) for T in (2, 4, 8, 16, 32, 64, 128)]


FOLD_SHAPES = [(T, E) for T in (64, 128, 256) for E in (2, 3)]  # as fold_team_shape() in zk_kernels.hpp


def lanes_ok(T, E, pad, real_bytes):
    """as row_lanes_ok() in zk_kernels.hpp"""
    N, tpb = T * E, max(T, 256) // T
    return pad and E % 5 != 0 and T % 64 == 0 and T <= 1024 and 2 * tpb * N * 2 * real_bytes <= 100 * 1024


def bs(T):
    return max(256, T)


def targs(kind, T, E, pad, lift=False):
    """template arguments of a kernel instance after its real type: row
    kernels (T, E[, PAD]), column kernels (T, E[, LIFTSYM[, PAD]]); the padded
    flag is written only where it differs from its default, E % 3 == 0"""
    out = [str(T), str(E)]
    odd = pad != (E % 3 == 0)
    if kind == "col" and (lift or odd):
        out.append("true" if lift else "false")
    if odd:
        out.append("true" if pad else "false")
    return ", ".join(out)

for kind in ("row", "col"):
    for real, tag in (("double", "f64"), ("float", "f32")):
        lines = [f"// zk_batch_{kind}_{tag}.hip -- batched {kind}-pass kernel instances ({real} transforms);",
                 "// written by gen_batch_units.py.",
                 '#include "zk_kernels.hpp"', "", "namespace zk {", "", "template <>",
                 f"const void *batch_{kind}_kernel<{real}>(int T, int E, bool pad) {{"]
        for T, E, pad in SHAPES:
            ta = targs(kind, T, E, pad)
            lines.append(f"  if (T == {T} && E == {E} && pad == {'true' if pad else 'false'}) return reinterpret_cast<const void *>(&{kind}_kernel_batch<{real}, {ta}>);")
        lines += ["  return nullptr;", "}", "",
                  "template <>",
                  f"hipError_t launch_batch_{kind}<{real}>(int T, int E, bool pad, dim3 grid, hipStream_t s, const {'RowArgs' if kind == 'row' else 'ColArgs'}<{real}> *args,",
                  "                                   const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph) {"]
        for T, E, pad in SHAPES:
            ta = targs(kind, T, E, pad)
            lines.append(f"  if (T == {T} && E == {E} && pad == {'true' if pad else 'false'}) {{")
            lines.append(f"    hipLaunchKernelGGL(({kind}_kernel_batch<{real}, {ta}>), grid, dim3({bs(T)}), 0, s, args, items, tile0, first0, sched0, ph);")
            lines.append("    return hipGetLastError();")
            lines.append("  }")
        lines += ["  return hipErrorInvalidValue;", "}", ""]
        if kind == "col":  # the lift_sym variant, base-length shapes only
            lines += ["template <>",
                      f"hipError_t launch_batch_col_lift<{real}>(int T, int E, dim3 grid, hipStream_t s, const ColArgs<{real}> *args,",
                      "                                        const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph) {"]
            for T, E, pad in SHAPES:
                if pad:
                    continue
                lines.append(f"  if (T == {T} && E == {E}) {{")
                lines.append(f"    hipLaunchKernelGGL((col_kernel_batch<{real}, {targs('col', T, E, pad, True)}>), grid, dim3({bs(T)}), 0, s, args, items, tile0, first0, sched0, ph);")
                lines.append("    return hipGetLastError();")
                lines.append("  }")
            lines += ["  return hipErrorInvalidValue;", "}", ""]
            # fold teams: kMaxFolds teams of T threads, one column per block
            lines += ["template <>",
                      f"hipError_t launch_batch_col_folds<{real}>(int T, int E, dim3 grid, hipStream_t s, const ColArgs<{real}> *args,",
                      "                                         const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph) {"]
            for T, E in FOLD_SHAPES:
                lines.append(f"  if (T == {T} && E == {E}) {{")
                lines.append(f"    hipLaunchKernelGGL((col_kernel_folds<{real}, {T}, {E}>), grid, dim3(kMaxFolds * {T}), 0, s, args, items, tile0, first0, sched0, ph);")
                lines.append("    return hipGetLastError();")
                lines.append("  }")
            lines += ["  return hipErrorInvalidValue;", "}", ""]
        if kind == "row":  # the permuted-layout form of the padded shapes that have one
            rb = 8 if real == "double" else 4
            lanes = [(T, E) for T, E, pad in SHAPES if lanes_ok(T, E, pad, rb)]
            lines += ["template <>", f"const void *lanes_row_kernel<{real}>(int T, int E) {{"]
            for T, E in lanes:
                lines.append(f"  if (T == {T} && E == {E}) return reinterpret_cast<const void *>(&row_kernel_batch<{real}, {T}, {E}, true, true>);")
            lines += ["  return nullptr;", "}", "",
                      "template <>",
                      f"hipError_t launch_lanes_row<{real}>(int T, int E, dim3 grid, hipStream_t s, const RowArgs<{real}> *args,",
                      "                                   const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph) {"]
            for T, E in lanes:
                lines.append(f"  if (T == {T} && E == {E}) {{")
                lines.append(f"    hipLaunchKernelGGL((row_kernel_batch<{real}, {T}, {E}, true, true>), grid, dim3({bs(T)}), 0, s, args, items, tile0, first0, sched0, ph);")
                lines.append("    return hipGetLastError();")
                lines.append("  }")
            lines += ["  return hipErrorInvalidValue;", "}", ""]
        lines += ["}  // namespace zk", ""]
        with open(os.path.join(HERE, f"zk_batch_{kind}_{tag}.hip"), "w") as f:
            f.write("\n".join(lines))
