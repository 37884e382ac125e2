// zk_plan.hpp -- host planner: turns order M into row programs and column tasks.
//
// Notation (base band spectra unless marked "mixed"):
//   eta^<l>  nested dealiased powers, eta^<1> = eta, eta^<l> = P(eta, eta^<l-1>)
//   Phi^(m)  surface-potential terms: Phi^(0) = psi,
//            Phi^(m) = -sum_{l=1..m} (1/l!) P(eta^<l>, L_l Phi^(m-l))   (Sec. 4.2)
//   W_j      = L_1 Phi^(j) + sum_{l=1..j} (1/l!) P(eta^<l>, L_{l+1} Phi^(j-l))
//   G_0 = W_0, G_1 = W_1 - P(eta_x, psi_x) - P(eta_y, psi_y),
//   G_j = W_j + P(S, W_{j-2}), S = P(eta_x, eta_x) + P(eta_y, eta_y)     (j >= 2)
//   G^[M] = sum_{j<M} eps^j G_j   (Sec. 3.2, eq:G1, eq:G2, eq:dno_truncated)
// Level r (1 <= r <= M-1) is one row pass producing the products of degree r
// (PHI_r -> Phi^(r), WP_r -> the product part of W_r, EP -> eta^<r+1>, S, GX
// for the G-only terms) and one column pass folding them and lifting what
// level r+1 needs.  The S * W terms of all orders are gathered into one
// product P(S, V), V = sum_{i<=M-3} eps^(i+2) W_i, at the last level.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "zk_program.hpp"

namespace zk {

enum LaunchKind : int { L_ROW_PAD = 0, L_ROW_BASE = 1, L_COL_PAD = 2, L_COL_BASE = 3, L_PARSEVAL = 4 };

struct Launch {
  int kind;
  int first, count;  // program or task range; for L_PARSEVAL: base ids a, b (c, d in c2, d2)
                     // a column launch with c2 = 1 applies its outputs' lift_sym (depth lift);
                     // d2 = kMaxFolds marks one a single grid may run with fold teams
  int c2, d2;
  double bytes;  // algorithmic HBM bytes of the launch (fields read + written once each)
  double flops;  // FFT flops of the launch, 5 N log2 N per complex transform of length N
};

struct PlanParams {
  int nx, ny, M;
  double Lx, Ly, depth, g;
  double eps;
  bool taper, filt;
  int real_bytes = 8;  // bytes of one real in the transforms (8: FP64, 4: FP32)
};

struct Plan {
  std::vector<RowOp> ops;
  std::vector<RowProg> progs;
  std::vector<ColTerm> terms;
  std::vector<ColOut> outs;
  std::vector<ColTask> tasks;
  int nmix = 0, nbase = 0;

  // launch sequences
  std::vector<Launch> dtn, rhs, ham;
  std::vector<Launch> step_entry;     // physical -> spectral state U[0], lifts for stage 1
  std::vector<Launch> step_body[2];   // one RK4 step from U[p] to U[1-p] (no trailing lift)
  std::vector<Launch> step_lift[2];   // lifts of U[p] for the next step's stage 1
  std::vector<Launch> step_exit[2];   // U[p] -> physical
  int chk_e[2], chk_p[2];             // base ids of U[p] (finite check)
  // Pieces for stepping with an externally supplied DtN (learned closure):
  // Exact-linear Adams-Bashforth 2 (Sec. 3.4): one RHS per step, state U[p] -> U[1-p],
  // forcing F_n stored in F[p]; the first step of a call is the IF-Euler bootstrap.
  std::vector<Launch> ab2_first[2];
  std::vector<Launch> ab2_body[2];
  // Inverse DNO map (eq:psi_inverse): (eta, v) -> psi; entry seeds psi = G0^{-1} v,
  // each iteration psi <- psi + G0^{-1} (v - G^[M] psi), exit writes psi.
  std::vector<Launch> inv_entry, inv_iter, inv_exit;
  // Bulk velocity (Alg. ComputeVolumeVelFrom2D): lift_phi stores the tapered
  // first-order potential on the flat plane; depth_chunk[r] (1 <= r <=
  // depth_chunk_max) lifts r layers, whose depths the column args carry, in
  // one column and one row launch and writes (u, v, w) of layer i to planes
  // 3i, 3i+1, 3i+2 of output slot 0.
  std::vector<Launch> lift_phi;
  std::vector<Launch> depth_chunk[kMaxChunkLayers + 1];
  int depth_chunk_max = 0;
  std::vector<Launch> rhs_g;   // eta, psi, G (LDP slots 0, 1, 2) -> eta_t = P_B G, psi_t
  std::vector<Launch> filter;  // eta, psi -> A eta, A psi (the state filter alone)
};

// Every launch sequence of a plan (for annotation, validation and dumps).
std::vector<std::vector<Launch> *> plan_sequences(Plan &p);

// Build the full plan (host only; deterministic).  Throws std::runtime_error
// on an internal inconsistency.
Plan build_plan(const PlanParams &pp, double dt);

// Number of ops etc. are small; this validates every id and range against
// the plan's own sizes (used by the host before any launch and by the tests).
std::string validate_plan(const Plan &p, int rows_pad, int rows_base);

}  // namespace zk
