"""Build libzk.so (gfx950) in-tree from csrc/ with hipcc.

Every .hip unit and the HIP host unit are compiled in parallel into
_build/, then linked into paper_2608_25203_amd/libzk.so.  Flags:
  --offload-arch=gfx950                 CDNA4 code objects only
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                        no packed FP32 instructions
  -mllvm -simplifycfg-sink-common=false keeps the per-register-set switch
                                        cases of the row program interpreter
                                        apart, so register arrays stay in
                                        registers instead of private memory
  -mllvm -amdgpu-kernarg-preload-count=5
                                        the first kernel arguments arrive in
                                        SGPRs (no dependent kernarg load)
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libzk.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_UNITS = ["zk_reduce.hip", "zk_bc.hip", "zk_cnn.hip", "zk_closure.hip", "zk_batch_row_f64.hip", "zk_batch_row_f32.hip", "zk_batch_col_f64.hip",
             "zk_batch_col_f32.hip", "zk_persist.hip"]
HIP_HOST_UNITS = ["zk_api.cpp", "zk_cnn_api.cpp", "zk_closure_api.cpp", "zk_batch.cpp"]
CXX_UNITS = ["zk_plan.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-simplifycfg-sink-common=false",
             # the first kernel arguments (the record and item pointers, a
             # single grid's record index, first item and schedule table)
             # arrive preloaded in SGPRs: no dependent scalar load before a
             # block's first work
             "-mllvm", "-amdgpu-kernarg-preload-count=5"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(jobs=None, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    cmds = []
    objs = []
    for u in HIP_UNITS:
        o = os.path.join(BUILD, u + ".o")
        cmds.append([HIPCC] + HIP_FLAGS + COMMON + ["-c", os.path.join(CSRC, u), "-o", o])
        objs.append(o)
    for u in HIP_HOST_UNITS:
        o = os.path.join(BUILD, u + ".o")
        cmds.append([HIPCC] + HIP_FLAGS + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, u), "-o", o])
        objs.append(o)
    for u in CXX_UNITS:
        o = os.path.join(BUILD, u + ".o")
        cmds.append(["g++"] + COMMON + ["-c", os.path.join(CSRC, u), "-o", o])
        objs.append(o)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        for cmd, _ in zip(cmds, ex.map(_run, cmds)):
            if verbose:
                print(" ".join(cmd[:1] + cmd[-3:]), flush=True)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


def build_plan_check():
    """Host-only planner check binary (no GPU needed): validates every plan."""
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "zk_plan_check")
    _run(["g++"] + COMMON + [os.path.join(CSRC, "zk_plan.cpp"), os.path.join(CSRC, "zk_plan_check.cpp"),
                             "-o", exe])
    return exe


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
