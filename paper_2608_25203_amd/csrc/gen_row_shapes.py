"""Writes zk_row_shapes.hpp: the distinct operation sequences ("shapes") of the
planner's row programs, which the padded row kernels compile as straight-line
code (register sets fixed at compile time, no interpreter loop).  A shape is
the sequence of (code, a, b, c) of a program's RowOps; field ids, flags and
coefficients stay in the op records.  Programs whose shape is not listed run
in the interpreter, so a stale table costs speed, never correctness.
Programs longer than MAX_LEN operations are left out.

Builds the host plan dump (zk_plan.cpp + zk_plan_check.cpp, g++) in a
temporary directory and collects the row programs of every sequence for
HOS orders 1 to 8 over a spread of grids and options.  Run from any
directory; the header is committed, this script regenerates it."""
import json
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROW_KINDS = (0,)  # L_ROW_PAD: the padded row passes, the only ones compiled per shape
RECORDS = ("nmix", "nbase", "depth_chunk_max", "ops", "progs", "terms", "outs", "tasks", "chk")
GRIDS = ((64, 64), (64, 1), (96, 48))
# Longer programs (from 25 operations: HOS order 6's longest level and beyond)
# stay interpreted: compiled, their register peak crosses an occupancy step.
MAX_LEN = 22
OPTIONS = ((1.0, 1, 1, 1.0), (0.85, 0, 0, 0.01), (1.0, 1, 0, 0.05))


def build_dump(out_dir):
    exe = os.path.join(out_dir, "zk_plan_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", HERE, os.path.join(HERE, "zk_plan.cpp"),
                    os.path.join(HERE, "zk_plan_check.cpp"), "-o", exe], check=True)
    return exe


def program_shapes(plan):
    """the shapes of every row program that a row launch of the plan runs"""
    out = set()
    for key, seq in plan.items():
        if key in RECORDS:
            continue
        for kind, first, count, _, _ in seq:
            if kind in ROW_KINDS:
                for pi in range(first, first + count):
                    op0, nop = plan["progs"][pi]
                    if nop <= MAX_LEN:
                        out.add(tuple(tuple(o[:4]) for o in plan["ops"][op0:op0 + nop]))
    return out


def collect(exe):
    shapes = set()
    for M in range(1, 9):
        for nx, ny in GRIDS:
            for eps, taper, filt, dt in OPTIONS:
                txt = subprocess.run([exe, str(nx), str(ny), str(M), repr(eps), str(taper), str(filt), repr(dt)],
                                     capture_output=True, text=True, check=True).stdout
                shapes |= program_shapes(json.loads(txt))
    return sorted(shapes, key=lambda s: (len(s), s))


def word(op):
    code, a, b, c = op
    return code | a << 8 | b << 16 | c << 24


def header(shapes):
    n, mx = len(shapes), max(len(s) for s in shapes)
    lines = ["// zk_row_shapes.hpp -- operation sequences of the planner's row programs that",
             "// the padded row kernels compile as straight-line code; written by",
             "// gen_row_shapes.py.  Op word: code | a << 8 | b << 16 | c << 24 (RowOp fields).",
             "#pragma once",
             "#include <stdint.h>",
             "",
             "namespace zk {",
             "",
             f"constexpr int kRowShapes = {n};",
             f"constexpr int kRowShapeMaxLen = {mx};",
             "constexpr int kRowShapeLen[kRowShapes] = {" + ", ".join(str(len(s)) for s in shapes) + "};",
             "constexpr uint32_t kRowShapeOps[kRowShapes][kRowShapeMaxLen] = {"]
    for s in shapes:
        lines.append("    {" + ", ".join(f"0x{word(o):08x}u" for o in s) + "},")
    lines += ["};", "", "}  // namespace zk", ""]
    return "\n".join(lines)


def main():
    with tempfile.TemporaryDirectory() as d:
        shapes = collect(build_dump(d))
    with open(os.path.join(HERE, "zk_row_shapes.hpp"), "w") as f:
        f.write(header(shapes))
    print(f"{len(shapes)} row program shapes")


if __name__ == "__main__":
    main()
