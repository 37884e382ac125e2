// zk_ctx_internal.hpp -- the context behind the zk_* ABI, shared with the
// closure driver (zk_closure.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "zk_kernels.hpp"
#include "zk_plan.hpp"

struct zk_ctx {
  zk::PlanParams pp{};
  int precision = 64;
  int check = 1;
  std::string err;

  zk::Plan plan;
  double plan_dt = NAN;
  bool have_plan = false;
  bool dirty = true;  // schedules must be (re)uploaded

  // binding
  char *ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  bool bound = false;

  // workspace layout (byte offsets)
  size_t off_tw[4] = {0, 0, 0, 0};  // row pad, row base, col pad, col base
  size_t off_ops = 0, off_progs = 0, off_terms = 0, off_outs = 0, off_tasks = 0;
  size_t off_rargs = 0, off_cargs = 0, off_iprog = 0, off_itask = 0;
  int integrator = 0;     // ZK_INTEGRATOR_RK4 or ZK_INTEGRATOR_IFAB2
  int bc = 0;             // ZK_BC_PERIODIC or ZK_BC_REFLECT
  int unx = 0, uny = 0;   // caller's grid (the internal grid is doubled for walls)
  double uLx = 0, uLy = 0;
  size_t off_ext = 0;     // four doubled fields (walls only)
  size_t off_ifsym = 0;   // IF-AB2 coefficient table (0 when unused)
  size_t off_layer = 0;   // (C, S) of one depth layer per band element
  double ifsym_dt = NAN;  // dt the table holds
  int tuneT[2][2] = {{0, 0}, {0, 0}};  // [row][pad] autotuned threads per transform (0: default)
  int row_fft = 0;
  int row_programs = 1;  // ZK_OPT_ROW_PROGRAMS                      // ZK_OPT_ROW_FFT
  size_t off_red = 0, off_cmax = 0, off_sym = 0, off_fx = 0, off_fy = 0, off_base = 0, off_mix = 0, total = 0;
  long long base_stride = 0, mix_stride = 0;
  size_t sched_cap[5] = {0, 0, 0, 0, 0};  // capacities (elements) reserved for the schedules

  // optional per-kernel timing (ZK_OPT_PROFILE)
  struct Rec {
    int kind;
    double bytes, flops;
    hipEvent_t a, b;
  };
  bool prof = false;
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double st_ms[5] = {0, 0, 0, 0, 0}, st_bytes[5] = {0, 0, 0, 0, 0}, st_flops[5] = {0, 0, 0, 0, 0};
  long long st_n[5] = {0, 0, 0, 0, 0};
  ~zk_ctx() {
    for (auto &r : pending) {
      hipEventDestroy(r.a);
      hipEventDestroy(r.b);
    }
    for (auto e : pool) hipEventDestroy(e);
  }
};


namespace zk {

// Caller (or workspace) fields a launch sequence reads and writes: input
// slots 0..2 for OP_LDP, output slots 0..1 for OP_STP.
struct Phys {
  const double *in0 = nullptr, *in1 = nullptr, *in2 = nullptr;
  double *out0 = nullptr, *out1 = nullptr;
};

// Default team shape of a pass: T threads per transform, first-pass radix E,
// and the number of 256-thread blocks covering the pass's rows or columns.
struct TeamShape {
  int T, E, blocks;
};
TeamShape ctx_team(const zk_ctx *c, bool row, bool pad);
// Argument records of the context's passes (pointers into its workspace).
template <typename real>
RowArgs<real> ctx_row_args(const zk_ctx *c, bool pad, const Phys &ph, int prog0);
template <typename real>
ColArgs<real> ctx_col_args(const zk_ctx *c, bool pad, int task0);
// Build and upload the plan for step size dt (no-op if current).
int ctx_upload(zk_ctx *c, double dt);

// Validate the call, bind the device and make sure the schedules are uploaded
// (dt of the last zk_step, or the default schedule).
int ctx_prepare(zk_ctx *c);
// Enqueue one launch sequence of the context's plan on its stream.
int ctx_run(zk_ctx *c, const std::vector<Launch> &seq, const Phys &ph);

}  // namespace zk
