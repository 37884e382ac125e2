// zk_plan_check.cpp -- host-only tool: builds a plan, validates it and dumps it
// as JSON (used by the CPU tests to check the planner without a GPU).
//   zk_plan_check nx ny M eps taper filt dt
#include <cstdio>
#include <cstdlib>
#include <string>

#include "zk_plan.hpp"

using namespace zk;

static void dump_seq(const char *name, const std::vector<Launch> &s, bool last) {
  std::printf("\"%s\": [", name);
  for (size_t i = 0; i < s.size(); ++i)
    std::printf("%s[%d,%d,%d,%d,%d]", i ? "," : "", s[i].kind, s[i].first, s[i].count, s[i].c2, s[i].d2);
  std::printf("]%s\n", last ? "" : ",");
}

int main(int argc, char **argv) {
  if (argc != 8) {
    std::fprintf(stderr, "usage: %s nx ny M eps taper filt dt\n", argv[0]);
    return 2;
  }
  PlanParams pp{};
  pp.nx = std::atoi(argv[1]);
  pp.ny = std::atoi(argv[2]);
  pp.M = std::atoi(argv[3]);
  pp.Lx = pp.Ly = 1.0;
  pp.depth = 0.0;
  pp.g = 9.81;
  pp.eps = std::atof(argv[4]);
  pp.taper = std::atoi(argv[5]) != 0;
  pp.filt = std::atoi(argv[6]) != 0;
  const double dt = std::atof(argv[7]);
  Plan p;
  try {
    p = build_plan(pp, dt);
  } catch (const std::exception &e) {
    std::fprintf(stderr, "plan error: %s\n", e.what());
    return 1;
  }
  const std::string v = validate_plan(p, 3 * pp.ny / 2, pp.ny);
  if (!v.empty()) {
    std::fprintf(stderr, "validation: %s\n", v.c_str());
    return 1;
  }
  std::printf("{\"nmix\": %d, \"nbase\": %d, \"depth_chunk_max\": %d,\n", p.nmix, p.nbase, p.depth_chunk_max);
  std::printf("\"ops\": [");
  for (size_t i = 0; i < p.ops.size(); ++i) {
    const RowOp &o = p.ops[i];
    std::printf("%s[%d,%d,%d,%d,%d,%d,%d,%d,%.17g]", i ? "," : "", o.code, o.a, o.b, o.c, o.fa, o.fla, o.fb, o.flb,
                o.coef);
  }
  std::printf("],\n\"progs\": [");
  for (size_t i = 0; i < p.progs.size(); ++i) std::printf("%s[%d,%d]", i ? "," : "", p.progs[i].op0, p.progs[i].nop);
  std::printf("],\n\"terms\": [");
  for (size_t i = 0; i < p.terms.size(); ++i)
    std::printf("%s[%d,%u,%.17g]", i ? "," : "", p.terms[i].src, p.terms[i].sym, p.terms[i].coef);
  std::printf("],\n\"outs\": [");
  for (size_t i = 0; i < p.outs.size(); ++i)
    std::printf("%s[%d,%d,%d,%d,%.17g,%u]", i ? "," : "", p.outs[i].dst_base, p.outs[i].dst_mixed, p.outs[i].t0,
                p.outs[i].nt, p.outs[i].lift_coef, p.outs[i].lift_sym);
  std::printf("],\n\"tasks\": [");
  for (size_t i = 0; i < p.tasks.size(); ++i)
    std::printf("%s[[%d,%d,%d],[%u,%u,%u],[%.17g,%.17g,%.17g],%d,%d]", i ? "," : "", p.tasks[i].fwd[0],
                p.tasks[i].fwd[1], p.tasks[i].fwd[2], p.tasks[i].fwd_sym[0], p.tasks[i].fwd_sym[1],
                p.tasks[i].fwd_sym[2], p.tasks[i].fwd_coef[0], p.tasks[i].fwd_coef[1], p.tasks[i].fwd_coef[2],
                p.tasks[i].o0, p.tasks[i].no);
  std::printf("],\n\"chk\": [%d,%d,%d,%d],\n", p.chk_e[0], p.chk_p[0], p.chk_e[1], p.chk_p[1]);
  dump_seq("dtn", p.dtn, false);
  dump_seq("rhs", p.rhs, false);
  dump_seq("ham", p.ham, false);
  dump_seq("step_entry", p.step_entry, false);
  dump_seq("step_body0", p.step_body[0], false);
  dump_seq("step_body1", p.step_body[1], false);
  dump_seq("step_lift0", p.step_lift[0], false);
  dump_seq("step_lift1", p.step_lift[1], false);
  dump_seq("step_exit0", p.step_exit[0], false);
  dump_seq("step_exit1", p.step_exit[1], false);
  dump_seq("rhs_g", p.rhs_g, false);
  dump_seq("filter", p.filter, false);
  dump_seq("ab2_first0", p.ab2_first[0], false);
  dump_seq("ab2_first1", p.ab2_first[1], false);
  dump_seq("ab2_body0", p.ab2_body[0], false);
  dump_seq("ab2_body1", p.ab2_body[1], false);
  dump_seq("inv_entry", p.inv_entry, false);
  dump_seq("inv_iter", p.inv_iter, false);
  dump_seq("inv_exit", p.inv_exit, false);
  dump_seq("lift_phi", p.lift_phi, false);
  for (int r = 1; r <= p.depth_chunk_max; ++r)
    dump_seq(("depth_chunk" + std::to_string(r)).c_str(), p.depth_chunk[r], r == p.depth_chunk_max);
  std::printf("}\n");
  return 0;
}
