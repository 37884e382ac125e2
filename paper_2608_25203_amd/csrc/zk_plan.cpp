// zk_plan.cpp -- host planner (pure C++; no device code).
#include "zk_plan.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <stdexcept>
#include <utility>

namespace zk {
namespace {

constexpr int kMaxM = 8;

struct Fac {  // a factor of a product: mixed field id and x-derivative flag
  int f;
  uint8_t fl;
  bool operator==(const Fac &o) const { return f == o.f && fl == o.fl; }
  bool operator<(const Fac &o) const { return f < o.f || (f == o.f && fl < o.fl); }
};

struct Prod {
  Fac a, b;
  int out;  // logical output index inside the program
  double coef;
};

struct TermSpec {
  int src;
  uint32_t sym;
  double coef;
};

struct OutSpec {
  int dst_base = -1, dst_mixed = -1;
  std::vector<TermSpec> terms;
  double lift_coef = 1.0;
  uint32_t lift_sym = 0;
};

struct FoldSpec {
  int fwd;
  uint32_t sym;
  double coef;
};

struct TaskSpec {
  int fwd = -1;  // first fold
  uint32_t fwd_sym = 0;
  double fwd_coef = 1.0;
  std::vector<FoldSpec> more;  // further folds summed into the same X
  std::vector<OutSpec> outs;
};

class Builder {
 public:
  explicit Builder(const PlanParams &pp) : pp_(pp) {
    M = pp.M;
    // a 1D grid (ny = 1) is not padded along y: its products have ky = 0 only
    const double N = (double)pp.nx * pp.ny;
    const double Np = (1.5 * pp.nx) * (pp.ny > 1 ? 1.5 * pp.ny : 1.0);
    inv_n = 1.0 / N;
    fold = N / Np;
  }

  Plan P;
  int M;
  double inv_n, fold;

  int mix() { return P.nmix++; }
  int base() { return P.nbase++; }

  // ---- row programs --------------------------------------------------------
  int prog_begin() {
    P.progs.push_back({(int32_t)P.ops.size(), 0});
    return (int)P.progs.size() - 1;
  }
  void op(uint8_t code, uint8_t a, uint8_t b, uint8_t c, int fa, uint8_t fla, int fb, uint8_t flb, double coef) {
    RowOp o{};
    o.code = code;
    o.a = a;
    o.b = b;
    o.c = c;
    o.fla = fla;
    o.flb = flb;
    o.fa = fa;
    o.fb = fb;
    o.coef = coef;
    P.ops.push_back(o);
    P.progs.back().nop++;
  }
  void ld2(Fac x, int y_f, uint8_t y_fl) { op(OP_LD2, 0, 0, 0, x.f, x.fl, y_f, y_fl, 0.0); }
  void mac(int out, uint8_t x, uint8_t y, double c) { op(OP_MAC, (uint8_t)(RS_O0 + out), x, y, -1, 0, -1, 0, c); }

  // One program computing sum-of-products outputs (at most 3) and storing
  // them to the mixed fields outf[].  Products are grouped by a held factor,
  // greedily the factor shared by the most products; the groups' factors
  // and their partners form one load stream, [x1, y11, y12, ..., x2, y21,
  // ...], loaded two at a time, so a group's last partner may share its
  // transform with the next group's factor.  A holds the current group's
  // factor while partners arrive in later transforms.
  int product_program(std::vector<Prod> prods, const std::vector<int> &outf) {
    if (outf.empty() || outf.size() > 3) throw std::runtime_error("program outputs");
    const int pg = prog_begin();
    op(OP_ZERO, RS_O0, 0, 0, -1, 0, -1, 0, 0.0);  // clears all three outputs
    struct Group {
      Fac x;
      std::vector<Prod> partners, self;  // partners: x is .a
    };
    std::vector<Group> groups;
    while (!prods.empty()) {
      std::map<Fac, int> cnt;
      for (auto &p : prods) {
        cnt[p.a]++;
        if (!(p.b == p.a)) cnt[p.b]++;
      }
      Fac x = prods[0].a;
      int best = -1;
      for (auto &kv : cnt)
        if (kv.second > best) {
          best = kv.second;
          x = kv.first;
        }
      // Prefer a partner of the previous group as the next held factor: the
      // partner goes last in that group and its load serves both roles.
      if (!groups.empty()) {
        int pbest = -1;
        for (auto &q : groups.back().partners) {
          auto it = cnt.find(q.b);
          if (it != cnt.end() && it->second > pbest) {
            pbest = it->second;
            x = q.b;
          }
        }
        if (pbest > 0) {
          auto &ps = groups.back().partners;
          std::stable_partition(ps.begin(), ps.end(), [&](const Prod &q) { return !(q.b == x); });
        }
      }
      Group g{x, {}, {}};
      std::vector<Prod> keep;
      for (auto &p : prods) {
        if (p.a == x && p.b == x) g.self.push_back(p);
        else if (p.a == x) g.partners.push_back(p);
        else if (p.b == x) g.partners.push_back({p.b, p.a, p.out, p.coef});
        else keep.push_back(p);
      }
      groups.push_back(g);
      prods.swap(keep);
    }
    struct Item {
      Fac f;
      int group, partner;  // partner = -1: the group's held factor
      int also_hold;       // a partner that is also the next group's held factor, or -1
    };
    std::vector<Item> items;
    for (int gi = 0; gi < (int)groups.size(); ++gi) {
      const bool shared = !items.empty() && items.back().partner >= 0 && items.back().group == gi - 1 &&
                          items.back().f == groups[gi].x;
      if (shared) items.back().also_hold = gi;
      else items.push_back({groups[gi].x, gi, -1, -1});
      for (int k = 0; k < (int)groups[gi].partners.size(); ++k)
        items.push_back({groups[gi].partners[k].b, gi, k, -1});
    }
    int in_a = -1;                // group whose factor A holds
    int hold_group = -1, hold_reg = -1;  // a factor loaded in this transform's U or V
    for (size_t i = 0; i < items.size(); i += 2) {
      const bool two = i + 1 < items.size();
      ld2(items[i].f, two ? items[i + 1].f.f : -1, two ? items[i + 1].f.fl : 0);
      hold_group = -1;
      for (size_t j = i; j < i + (two ? 2 : 1); ++j) {
        const Item &it = items[j];
        const uint8_t reg = j == i ? RS_U : RS_V;
        const Group &g = groups[it.group];
        if (it.partner >= 0) {
          const Prod &p = g.partners[it.partner];
          const uint8_t h = (hold_group == it.group) ? (uint8_t)hold_reg : RS_A;
          if (h == RS_A && in_a != it.group) throw std::runtime_error("product schedule lost its held factor");
          mac(p.out, h, reg, p.coef);
        }
        const int hg = it.partner < 0 ? it.group : it.also_hold;
        if (hg >= 0) {  // a group's factor: self products, keep it if partners follow
          for (auto &p : groups[hg].self) mac(p.out, reg, reg, p.coef);
          hold_group = hg;
          hold_reg = reg;
          bool later = false;
          for (size_t k = j + 1; k < items.size(); ++k)
            if (items[k].group == hg && k >= i + 2) later = true;
          if (later) {
            op(OP_MOV, RS_A, reg, 0, -1, 0, -1, 0, 0.0);
            in_a = hg;
          }
        }
      }
    }
    for (size_t k = 0; k < outf.size(); k += 2) {
      if (k + 1 < outf.size())
        op(OP_ST2, (uint8_t)(RS_O0 + k), (uint8_t)(RS_O0 + k + 1), 0, outf[k], 0, outf[k + 1], 0, 0.0);
      else
        op(OP_ST2, (uint8_t)(RS_O0 + k), RS_NONE, 0, outf[k], 0, -1, 0, 0.0);
    }
    return pg;
  }

  // ---- column tasks --------------------------------------------------------
  static bool same_terms(const std::vector<TermSpec> &a, const std::vector<TermSpec> &b) {
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i)
      if (a[i].src != b[i].src || a[i].sym != b[i].sym || a[i].coef != b[i].coef) return false;
    return true;
  }
  void add_tasks(const std::vector<TaskSpec> &ts) {
    for (auto &t : ts) {
      ColTask ct{};
      if (t.more.size() + 1 > (size_t)kMaxFolds) throw std::runtime_error("too many folds in a task");
      for (int f = 0; f < kMaxFolds; ++f) {
        ct.fwd[f] = -1;
        ct.fwd_sym[f] = 0;
        ct.fwd_coef[f] = 0.0;
      }
      ct.fwd[0] = t.fwd;
      ct.fwd_sym[0] = t.fwd_sym;
      ct.fwd_coef[0] = t.fwd_coef;
      for (size_t f = 0; f < t.more.size(); ++f) {
        ct.fwd[f + 1] = t.more[f].fwd;
        ct.fwd_sym[f + 1] = t.more[f].sym;
        ct.fwd_coef[f + 1] = t.more[f].coef;
      }
      // A lift whose terms equal those of an earlier store of the same task
      // becomes that output's lifted copy: one combination, both destinations
      // (the store keeps its place; lifts write mixed fields, which no term reads).
      std::vector<OutSpec> outs;
      for (const auto &o : t.outs) {
        bool merged = false;
        if (o.dst_base < 0 && o.dst_mixed >= 0)
          for (auto &m : outs)
            if (m.dst_mixed < 0 && m.dst_base >= 0 && same_terms(m.terms, o.terms)) {
              m.dst_mixed = o.dst_mixed;
              m.lift_coef = o.lift_coef;
              m.lift_sym = o.lift_sym;
              merged = true;
              break;
            }
        if (!merged) outs.push_back(o);
      }
      ct.o0 = (int32_t)P.outs.size();
      ct.no = (int32_t)outs.size();
      for (auto &o : outs) {
        ColOut co{};
        co.dst_base = o.dst_base;
        co.dst_mixed = o.dst_mixed;
        co.t0 = (int32_t)P.terms.size();
        co.nt = (int32_t)o.terms.size();
        co.lift_coef = o.lift_coef;
        co.lift_sym = o.lift_sym;
        for (auto &tm : o.terms) P.terms.push_back({tm.src, tm.sym, tm.coef});
        P.outs.push_back(co);
      }
      P.tasks.push_back(ct);
    }
  }
  Launch col_launch(int kind, const std::vector<TaskSpec> &ts) {
    Launch l{kind, (int)P.tasks.size(), (int)ts.size(), 0, 0, 0.0, 0.0};
    add_tasks(ts);
    return l;
  }
  OutSpec lift(int dst_mixed, std::vector<TermSpec> terms, uint32_t lift_sym = 0) {
    OutSpec o;
    o.dst_mixed = dst_mixed;
    o.terms = std::move(terms);
    o.lift_coef = inv_n;
    o.lift_sym = lift_sym;
    return o;
  }
  OutSpec store(int dst_base, std::vector<TermSpec> terms) {
    OutSpec o;
    o.dst_base = dst_base;
    o.terms = std::move(terms);
    return o;
  }
  TaskSpec fold_task(int fwd) {  // fold of a dealiased product
    TaskSpec t;
    t.fwd = fwd;
    t.fwd_sym = SYM_TAPER;
    t.fwd_coef = fold;
    return t;
  }

 private:
  PlanParams pp_;
};

double fact(int l) {
  double f = 1.0;
  for (int i = 2; i <= l; ++i) f *= i;
  return f;
}

}  // namespace

Plan build_plan(const PlanParams &pp, double dt) {
  if (pp.M < 1 || pp.M > kMaxM) throw std::runtime_error("M out of range");
  Builder B(pp);
  const int M = B.M;
  const double eps = pp.eps, g = pp.g;
  const uint32_t FILT = pp.filt ? SYM_FILT : 0u;
  auto epow = [&](int j) { return std::pow(eps, (double)j); };
  // Fields are stored in kref units so that the two real fields sharing one
  // complex FFT have comparable magnitudes: lifted L_l fields divided by
  // kref^l, eta and its powers multiplied by kref^l (dimensionless, like the
  // slopes), the W products divided by kref.  The factors are undone in the
  // product and fold coefficients.  kref = kNyq / 3, a fixed mid-band
  // wavenumber.
  const double kref = (pp.ny > 1 ? std::min(M_PI * pp.nx / pp.Lx, M_PI * pp.ny / pp.Ly) : M_PI * pp.nx / pp.Lx) / 3.0;
  auto kpow = [&](int l) { return std::pow(kref, (double)l); };

  // ---- field ids -------------------------------------------------------------
  const int mE = B.mix(), mEy = B.mix(), mP = B.mix(), mPy = B.mix();
  int mL[kMaxM + 2], mEP[kMaxM + 2], mLPhi[kMaxM + 2][kMaxM + 2];
  for (int l = 1; l <= M; ++l) mL[l] = B.mix();
  for (int l = 2; l <= M - 1; ++l) mEP[l] = B.mix();
  for (int m = 1; m <= M - 2; ++m)
    for (int l = 1; l <= M - m; ++l) mLPhi[m][l] = B.mix();
  const int mS = (M >= 3) ? B.mix() : -1;
  const int mV = (M >= 4) ? B.mix() : -1;
  const int mG = B.mix(), mN = B.mix();
  const int oPHI = B.mix(), oWP = B.mix(), oEP = B.mix(), oS = B.mix(), oGX = B.mix();
  const int mbA = B.mix(), mbB = B.mix();

  int bUE[2], bUP[2], bSE[2], bSP[2];
  for (int i = 0; i < 2; ++i) {
    bUE[i] = B.base();
    bUP[i] = B.base();
  }
  for (int i = 0; i < 2; ++i) {
    bSE[i] = B.base();
    bSP[i] = B.base();
  }
  const int bAE = B.base(), bAP = B.base(), bG = B.base(), bPT = B.base(), bV = B.base(), bPhi0 = B.base();
  int bFe[2], bFp[2];  // IF-AB2 forcing of the last two steps
  for (int i = 0; i < 2; ++i) {
    bFe[i] = B.base();
    bFp[i] = B.base();
  }
  int bPHI[kMaxM + 2], bWP[kMaxM + 2], bGX[kMaxM + 2];
  for (int r = 1; r <= M - 1; ++r) {
    bPHI[r] = B.base();
    bWP[r] = B.base();
    bGX[r] = B.base();
  }

  auto etapow = [&](int l) { return Fac{l == 1 ? mE : mEP[l], 0}; };
  auto lphi = [&](int m, int l) { return Fac{m == 0 ? mL[l] : mLPhi[m][l], 0}; };
  const bool hasGX1 = M >= 2;
  const bool hasGXlast = M >= 3;

  // ---- row programs of the levels (state independent) ------------------------
  std::vector<std::vector<int>> level_progs(M + 1);
  for (int r = 1; r <= M - 1; ++r) {
    // outputs of this level, in order
    std::vector<int> outs;  // mixed ids
    std::vector<std::vector<Prod>> pr;
    auto out_index = [&](int fid) {
      outs.push_back(fid);
      pr.emplace_back();
      return (int)outs.size() - 1;
    };
    const int iPHI = out_index(oPHI);
    const int iWP = out_index(oWP);
    const int iEP = (r + 1 <= M - 1) ? out_index(oEP) : -1;
    const int iGX = ((r == 1 && hasGX1) || (r == M - 1 && hasGXlast)) ? out_index(oGX) : -1;
    const int iS = (r == 1 && M >= 3) ? out_index(oS) : -1;
    for (int l = 1; l <= r; ++l) {
      pr[iPHI].push_back({etapow(l), lphi(r - l, l), 0, -1.0 / fact(l)});
      pr[iWP].push_back({etapow(l), lphi(r - l, l + 1), 0, 1.0 / fact(l)});
    }
    if (iEP >= 0) pr[iEP].push_back({Fac{mE, 0}, etapow(r), 0, 1.0});
    if (r == 1 && iGX >= 0) {
      pr[iGX].push_back({Fac{mE, FL_DX}, Fac{mP, FL_DX}, 0, -eps / kref});
      pr[iGX].push_back({Fac{mEy, 0}, Fac{mPy, 0}, 0, -eps});
    }
    if (iS >= 0) {
      pr[iS].push_back({Fac{mE, FL_DX}, Fac{mE, FL_DX}, 0, 1.0 / (kref * kref)});
      pr[iS].push_back({Fac{mEy, 0}, Fac{mEy, 0}, 0, 1.0});
    }
    if (r == M - 1 && hasGXlast) {
      if (M == 3) pr[iGX].push_back({Fac{mS, 0}, Fac{mL[1], 0}, 0, eps * eps * kpow(1)});
      else pr[iGX].push_back({Fac{mS, 0}, Fac{mV, 0}, 0, 1.0});
    }
    // group outputs by three: [PHI, WP, EP] [GX, S]; the last level, the
    // longest program, as [PHI, WP] [GX] for two programs per row
    const size_t grp = (r == M - 1 && M >= 3) ? 2 : 3;
    for (size_t k0 = 0; k0 < outs.size(); k0 += grp) {
      std::vector<int> of;
      std::vector<Prod> ps;
      for (size_t k = k0; k < outs.size() && k < k0 + grp; ++k) {
        of.push_back(outs[k]);
        for (auto p : pr[k]) {
          p.out = (int)(k - k0);
          ps.push_back(p);
        }
      }
      level_progs[r].push_back(B.product_program(ps, of));
    }
  }

  // Bernoulli program: o0 = |grad eta|^2, o1 = grad eta . grad psi, o2 = |grad psi|^2
  int bern_prog = B.prog_begin();
  B.op(OP_ZERO, RS_O0, 0, 0, -1, 0, -1, 0, 0.0);
  B.ld2(Fac{mE, FL_DX}, mP, FL_DX);
  B.mac(0, RS_U, RS_U, 1.0 / (kref * kref));
  B.mac(1, RS_U, RS_V, 1.0 / kref);
  B.mac(2, RS_V, RS_V, 1.0);
  B.ld2(Fac{mEy, 0}, mPy, 0);
  B.mac(0, RS_U, RS_U, 1.0);
  B.mac(1, RS_U, RS_V, 1.0);
  B.mac(2, RS_V, RS_V, 1.0);
  B.ld2(Fac{mG, 0}, -1, 0);
  B.op(OP_BERN, 0, 0, 0, -1, 0, -1, 0, eps);
  B.op(OP_ST2, RS_O0, RS_NONE, 0, mN, 0, -1, 0, 0.0);

  // entry / exit programs on the base grid
  const int entry_prog = B.prog_begin();
  B.op(OP_LDP, 0, 0, 0, 0, 0, 1, 0, 0.0);
  B.op(OP_ST2, RS_U, RS_V, 0, mbA, 0, mbB, 0, 0.0);
  const int exit2_prog = B.prog_begin();
  B.ld2(Fac{mbA, 0}, mbB, 0);
  B.op(OP_STP, RS_U, 0, 0, 0, 0, -1, 0, 0.0);
  B.op(OP_STP, RS_V, 0, 0, 1, 0, -1, 0, 0.0);
  const int exit1_prog = B.prog_begin();
  B.ld2(Fac{mbA, 0}, -1, 0);
  B.op(OP_STP, RS_U, 0, 0, 0, 0, -1, 0, 0.0);

  // entry of a third caller field (slot 2) on the base grid
  const int entry_g_prog = B.prog_begin();
  B.op(OP_LDP, 0, 0, 0, 2, 0, -1, 0, 0.0);
  B.op(OP_ST2, RS_U, RS_V, 0, mbA, 0, -1, 0, 0.0);

  auto row_launch = [&](int kind, const std::vector<int> &progs) {
    // programs of one launch must be contiguous
    for (size_t i = 1; i < progs.size(); ++i)
      if (progs[i] != progs[0] + (int)i) throw std::runtime_error("non-contiguous programs");
    return Launch{kind, progs[0], (int)progs.size(), 0, 0, 0.0, 0.0};
  };

  // ---- column task builders -----------------------------------------------------
  // lifts of the stage state (e, p) for level 1 (and G for M == 1)
  auto l0_tasks = [&](int e, int p, bool lift_g) {
    std::vector<TaskSpec> ts;
    auto one = [&](OutSpec o) {
      TaskSpec t;
      t.outs.push_back(std::move(o));
      ts.push_back(std::move(t));
    };
    one(B.lift(mE, {{e, 0, kref}}));
    one(B.lift(mEy, {{e, SYM_IKY, 1.0}}));
    one(B.lift(mP, {{p, 0, 1.0}}));
    one(B.lift(mPy, {{p, SYM_IKY, 1.0}}));
    for (int l = 1; l <= M; ++l) one(B.lift(mL[l], {{p, (uint32_t)l, 1.0 / kpow(l)}}));
    if (M == 1) {
      TaskSpec t;
      t.outs.push_back(B.store(bG, {{p, 1u, 1.0}}));
      if (lift_g) t.outs.push_back(B.lift(mG, {{p, 1u, 1.0}}));
      ts.push_back(std::move(t));
    }
    return ts;
  };
  // levels 1..M-1 for stage state (e, p); ends with G stored (and lifted)
  // The last level stores nothing but its PHI, WP and GX folds, which only G
  // uses: one task folds all three (each with its G coefficient) into X and
  // assembles G from X and the stored lower levels (and lifts it), in the
  // same launch.  Its launch is marked for fold teams (d2 = kMaxFolds): a
  // single grid runs it with one team per fold and per output, side by side
  // (a 512 x 512 grid has only 256 columns, one block per CU).
  auto last_level_g = [&](int p, bool lift_g) -> std::vector<TaskSpec> {
    const int r = M - 1;
    TaskSpec t;
    t.fwd = oPHI;
    t.fwd_sym = SYM_TAPER | 1u;
    t.fwd_coef = B.fold * epow(r);
    t.more.push_back({oWP, SYM_TAPER, B.fold * kref * epow(r)});
    if ((r == 1 && hasGX1) || (r == M - 1 && hasGXlast)) t.more.push_back({oGX, SYM_TAPER, B.fold});
    std::vector<TermSpec> tm{{p, 1u, 1.0}};
    for (int i = 1; i < r; ++i) {
      tm.push_back({bPHI[i], 1u, epow(i)});
      tm.push_back({bWP[i], 0u, epow(i)});
    }
    if (hasGX1 && r != 1) tm.push_back({bGX[1], 0u, 1.0});
    tm.push_back({-1, 0u, 1.0});
    t.outs.push_back(B.store(bG, tm));
    if (lift_g) t.outs.push_back(B.lift(mG, tm));
    return {t};
  };
  auto core = [&](std::vector<Launch> &seq, int e, int p, bool lift_g) {
    (void)e;
    for (int r = 1; r <= M - 1; ++r) {
      seq.push_back(row_launch(L_ROW_PAD, level_progs[r]));
      if (r == M - 1) {
        seq.push_back(B.col_launch(L_COL_PAD, last_level_g(p, lift_g)));
        seq.back().d2 = kMaxFolds;  // fold teams
        continue;
      }
      std::vector<TaskSpec> A;
      {
        TaskSpec t = B.fold_task(oPHI);
        t.outs.push_back(B.store(bPHI[r], {{-1, 0, 1.0}}));
        if (r <= M - 2)
          for (int l = 1; l <= M - r; ++l) t.outs.push_back(B.lift(mLPhi[r][l], {{-1, (uint32_t)l, 1.0 / kpow(l)}}));
        A.push_back(std::move(t));
      }
      {
        TaskSpec t = B.fold_task(oWP);
        t.fwd_coef *= kref;
        t.outs.push_back(B.store(bWP[r], {{-1, 0, 1.0}}));
        A.push_back(std::move(t));
      }
      if (r + 1 <= M - 1) {
        TaskSpec t = B.fold_task(oEP);
        t.outs.push_back(B.lift(mEP[r + 1], {{-1, 0, 1.0}}));
        A.push_back(std::move(t));
      }
      if (r == 1 && M >= 3) {
        TaskSpec t = B.fold_task(oS);
        t.outs.push_back(B.lift(mS, {{-1, 0, 1.0}}));
        A.push_back(std::move(t));
      }
      if ((r == 1 && hasGX1) || (r == M - 1 && hasGXlast)) {
        TaskSpec t = B.fold_task(oGX);
        t.outs.push_back(B.store(bGX[r], {{-1, 0, 1.0}}));
        A.push_back(std::move(t));
      }
      if (r == M - 2 && M >= 4) {
        std::vector<TermSpec> tm{{p, 1u, epow(2)}};
        for (int i = 1; i <= M - 3; ++i) {
          tm.push_back({bPHI[i], 1u, epow(i + 2)});
          tm.push_back({bWP[i], 0u, epow(i + 2)});
        }
        TaskSpec t;
        t.outs.push_back(B.lift(mV, tm));
        A.push_back(std::move(t));
      }
      seq.push_back(B.col_launch(L_COL_PAD, A));
    }
  };
  auto entry = [&](std::vector<Launch> &seq) {
    seq.push_back(row_launch(L_ROW_BASE, {entry_prog}));
    std::vector<TaskSpec> ts(2);
    ts[0].fwd = mbA;
    ts[0].outs.push_back(B.store(bUE[0], {{-1, 0, 1.0}}));
    ts[1].fwd = mbB;
    ts[1].outs.push_back(B.store(bUP[0], {{-1, 0, 1.0}}));
    seq.push_back(B.col_launch(L_COL_BASE, ts));
  };
  auto exit_seq = [&](std::vector<Launch> &seq, int a, int b) {
    std::vector<TaskSpec> ts(b >= 0 ? 2 : 1);
    ts[0].outs.push_back(B.lift(mbA, {{a, 0, 1.0}}));
    if (b >= 0) ts[1].outs.push_back(B.lift(mbB, {{b, 0, 1.0}}));
    seq.push_back(B.col_launch(L_COL_BASE, ts));
    seq.push_back(row_launch(L_ROW_BASE, {b >= 0 ? exit2_prog : exit1_prog}));
  };

  Plan &P = B.P;
  // zk_dtn
  entry(P.dtn);
  P.dtn.push_back(B.col_launch(L_COL_PAD, l0_tasks(bUE[0], bUP[0], false)));
  core(P.dtn, bUE[0], bUP[0], false);
  exit_seq(P.dtn, bG, -1);
  // zk_hamiltonian
  entry(P.ham);
  P.ham.push_back(B.col_launch(L_COL_PAD, l0_tasks(bUE[0], bUP[0], false)));
  core(P.ham, bUE[0], bUP[0], false);
  P.ham.push_back(Launch{L_PARSEVAL, bUP[0], bG, bUE[0], bUE[0], 0.0, 0.0});
  // zk_rhs
  entry(P.rhs);
  P.rhs.push_back(B.col_launch(L_COL_PAD, l0_tasks(bUE[0], bUP[0], true)));
  core(P.rhs, bUE[0], bUP[0], true);
  P.rhs.push_back(row_launch(L_ROW_PAD, {bern_prog}));
  {
    TaskSpec t = B.fold_task(mN);
    t.outs.push_back(B.store(bPT, {{bUE[0], 0, -g}, {-1, 0, 1.0}}));
    P.rhs.push_back(B.col_launch(L_COL_PAD, {t}));
  }
  exit_seq(P.rhs, bG, bPT);

  // zk_step: RK4 stages, state U[par] -> U[1 - par]
  entry(P.step_entry);
  P.step_entry.push_back(B.col_launch(L_COL_PAD, l0_tasks(bUE[0], bUP[0], true)));
  const double cnext[4] = {0.5 * dt, 0.5 * dt, dt, 0.0};
  const double wacc[4] = {1.0, 2.0, 2.0, 0.0};
  for (int par = 0; par < 2; ++par) {
    auto &seq = P.step_body[par];
    const int se[5] = {0, bUE[par], bSE[0], bSE[1], bSE[0]};
    const int sp[5] = {0, bUP[par], bSP[0], bSP[1], bSP[0]};
    const int ne[5] = {0, bSE[0], bSE[1], bSE[0], bUE[1 - par]};
    const int np[5] = {0, bSP[0], bSP[1], bSP[0], bUP[1 - par]};
    for (int s = 1; s <= 4; ++s) {
      core(seq, se[s], sp[s], true);
      seq.push_back(row_launch(L_ROW_PAD, {bern_prog}));
      TaskSpec tp = B.fold_task(mN), te;
      const double c = cnext[s - 1], w = wacc[s - 1];
      if (s < 4) {
        std::vector<TermSpec> ap{{se[s], 0, -g * w}, {-1, 0, w}};
        std::vector<TermSpec> ae{{bG, 0, w}};
        if (s > 1) {
          ap.push_back({bAP, 0, 1.0});
          ae.push_back({bAE, 0, 1.0});
        }
        const std::vector<TermSpec> pt{{bUP[par], 0, 1.0}, {se[s], 0, -g * c}, {-1, 0, c}};  // next stage psi
        const std::vector<TermSpec> et{{bUE[par], 0, 1.0}, {bG, 0, c}};                      // next stage eta
        tp.outs.push_back(B.store(bAP, ap));
        tp.outs.push_back(B.store(np[s], pt));
        te.outs.push_back(B.store(bAE, ae));
        te.outs.push_back(B.store(ne[s], et));
        if (M >= 2) {
          // The next stage's lifts in the same launch, each from the stage
          // combination itself (the tasks that need the folded N fold it
          // again): one launch instead of two.  (M = 1 stores G from psi in
          // its lift launch, which te's read of this stage's G forbids.)
          auto with = [](std::vector<TermSpec> tm, uint32_t sym, double f) {
            for (auto &x : tm) {
              x.sym |= sym;
              x.coef *= f;
            }
            return tm;
          };
          tp.outs.push_back(B.lift(mP, with(pt, 0, 1.0)));
          tp.outs.push_back(B.lift(mPy, with(pt, SYM_IKY, 1.0)));
          te.outs.push_back(B.lift(mE, with(et, 0, kref)));
          te.outs.push_back(B.lift(mEy, with(et, SYM_IKY, 1.0)));
          std::vector<TaskSpec> ts{tp, te};
          for (int l = 1; l <= M; l += 2) {
            TaskSpec tl = B.fold_task(mN);
            for (int m = l; m <= std::min(M, l + 1); ++m)
              tl.outs.push_back(B.lift(mL[m], with(pt, (uint32_t)m, 1.0 / kpow(m))));
            ts.push_back(tl);
          }
          seq.push_back(B.col_launch(L_COL_PAD, ts));
          continue;
        }
      } else {
        const double h = dt / 6.0;
        tp.outs.push_back(B.store(np[s], {{bUP[par], FILT, 1.0}, {bAP, FILT, h}, {se[s], FILT, -g * h}, {-1, FILT, h}}));
        te.outs.push_back(B.store(ne[s], {{bUE[par], FILT, 1.0}, {bAE, FILT, h}, {bG, FILT, h}}));
      }
      seq.push_back(B.col_launch(L_COL_PAD, {tp, te}));
      if (s < 4) seq.push_back(B.col_launch(L_COL_PAD, l0_tasks(ne[s], np[s], true)));
    }
    P.step_lift[par].push_back(B.col_launch(L_COL_PAD, l0_tasks(bUE[par], bUP[par], true)));
    exit_seq(P.step_exit[par], bUE[par], bUP[par]);
    P.chk_e[par] = bUE[par];
    P.chk_p[par] = bUP[par];
  }

  // ---- IF-AB2: F = (G^[M] psi - G0 psi, N); U <- A [E(dt) U + D(dt) F*] ----------
  {
    auto ifs = [&](int k) { return (uint32_t)(SYM_IF | (k << SYM_IF_SHIFT)) | FILT; };
    enum { IC = 0, IA = 1, IB = 2, IS = 3, IU = 4, IV = 5 };
    for (int first = 1; first >= 0; --first)
      for (int par = 0; par < 2; ++par) {
        auto &seq = first ? P.ab2_first[par] : P.ab2_body[par];
        const int e = bUE[par], p = bUP[par];
        core(seq, e, p, true);
        seq.push_back(row_launch(L_ROW_PAD, {bern_prog}));
        TaskSpec t = B.fold_task(mN);  // X = N (folded Bernoulli term)
        t.outs.push_back(B.store(bFe[par], {{bG, 0, 1.0}, {p, 1u, -1.0}}));
        t.outs.push_back(B.store(bFp[par], {{-1, 0, 1.0}}));
        const double w = first ? 1.0 : 1.5;  // F* = 3/2 F_n - 1/2 F_{n-1} (F_0 at the bootstrap)
        std::vector<TermSpec> te{{e, ifs(IC), 1.0}, {p, ifs(IA), 1.0},  {bG, ifs(IS), w},
                                 {p, ifs(IS) | 1u, -w}, {-1, ifs(IU), w}};
        std::vector<TermSpec> tp{{e, ifs(IB), -1.0}, {p, ifs(IC), 1.0}, {bG, ifs(IV), -w},
                                 {p, ifs(IV) | 1u, w},   {-1, ifs(IS), w}};
        if (!first) {
          te.push_back({bFe[1 - par], ifs(IS), -0.5});
          te.push_back({bFp[1 - par], ifs(IU), -0.5});
          tp.push_back({bFe[1 - par], ifs(IV), 0.5});
          tp.push_back({bFp[1 - par], ifs(IS), -0.5});
        }
        t.outs.push_back(B.store(bUE[1 - par], te));
        t.outs.push_back(B.store(bUP[1 - par], tp));
        seq.push_back(B.col_launch(L_COL_PAD, {t}));
      }
  }

  // ---- inverse DNO map ------------------------------------------------------------
  {
    P.inv_entry.push_back(row_launch(L_ROW_BASE, {entry_prog}));
    std::vector<TaskSpec> ts(2);
    ts[0].fwd = mbA;
    ts[0].outs.push_back(B.store(bUE[0], {{-1, 0, 1.0}}));
    ts[1].fwd = mbB;
    ts[1].outs.push_back(B.store(bV, {{-1, 0, 1.0}}));
    ts[1].outs.push_back(B.store(bUP[0], {{-1, SYM_INVG0, 1.0}}));
    P.inv_entry.push_back(B.col_launch(L_COL_BASE, ts));
    P.inv_entry.push_back(B.col_launch(L_COL_PAD, l0_tasks(bUE[0], bUP[0], false)));
    core(P.inv_iter, bUE[0], bUP[0], false);
    TaskSpec t;
    t.outs.push_back(B.store(bUP[0], {{bUP[0], 0, 1.0}, {bV, SYM_INVG0, 1.0}, {bG, SYM_INVG0, -1.0}}));
    P.inv_iter.push_back(B.col_launch(L_COL_PAD, {t}));
    P.inv_iter.push_back(B.col_launch(L_COL_PAD, l0_tasks(bUE[0], bUP[0], false)));
    exit_seq(P.inv_exit, bUP[0], -1);
  }

  // ---- bulk velocity at depth layers ----------------------------------------------
  {
    entry(P.lift_phi);
    std::vector<TaskSpec> ts(2);
    ts[0].outs.push_back(B.lift(mE, {{bUE[0], 0, kref}}));
    ts[1].outs.push_back(B.lift(mL[1], {{bUP[0], 1u, 1.0 / kpow(1)}}));
    P.lift_phi.push_back(B.col_launch(L_COL_PAD, ts));
    const int prod = B.product_program({{Fac{mE, 0}, Fac{mL[1], 0}, 0, 1.0}}, {oPHI});
    P.lift_phi.push_back(row_launch(L_ROW_PAD, {prod}));
    TaskSpec t = B.fold_task(oPHI);  // X = P(eta, G0 psi)
    t.outs.push_back(B.store(bPhi0, {{bUP[0], 0, 1.0}, {-1, 0, -eps}}));  // the taper comes with each layer
    P.lift_phi.push_back(B.col_launch(L_COL_PAD, {t}));
    // Chunks: every mixed field is free once Phi|0 is stored, three per layer.
    const int lc = std::min(kMaxChunkLayers, P.nmix / 3);
    P.depth_chunk_max = lc;
    for (int r = 1; r <= lc; ++r) {
      std::vector<TaskSpec> ts(r);
      for (int i = 0; i < r; ++i) {
        const uint32_t li = SYM_COUPLE | ((uint32_t)i << SYM_LAYER_SHIFT);
        ts[i].outs.push_back(B.lift(3 * i, {{bPhi0, 0, 1.0}}, SYM_LAYER_C | li));            // C Phi (d_x in the row pass)
        ts[i].outs.push_back(B.lift(3 * i + 1, {{bPhi0, 0, 1.0}}, SYM_LAYER_S | li));        // v = S Phi
        ts[i].outs.push_back(B.lift(3 * i + 2, {{bPhi0, SYM_IKY, 1.0}}, SYM_LAYER_C | li));  // w = i ky C Phi
      }
      Launch cl = B.col_launch(L_COL_BASE, ts);
      cl.c2 = 1;  // the lift_sym kernel variant
      P.depth_chunk[r].push_back(cl);
      std::vector<int> progs;
      for (int i = 0; i < r; i += 2) {
        progs.push_back(B.prog_begin());
        const int n2 = std::min(2, r - i);
        for (int j = i; j < i + n2; ++j) {
          B.ld2(Fac{3 * j, FL_DX}, 3 * j + 2, 0);
          B.op(OP_STP, RS_U, 0, 0, 0, 0, 3 * j, 0, 0.0);
          B.op(OP_STP, RS_V, 0, 0, 0, 0, 3 * j + 2, 0, 0.0);
        }
        B.ld2(Fac{3 * i + 1, 0}, n2 == 2 ? 3 * i + 4 : -1, 0);
        B.op(OP_STP, RS_U, 0, 0, 0, 0, 3 * i + 1, 0, 0.0);
        if (n2 == 2) B.op(OP_STP, RS_V, 0, 0, 0, 0, 3 * i + 4, 0, 0.0);
      }
      P.depth_chunk[r].push_back(row_launch(L_ROW_BASE, progs));
    }
  }

  // ---- stepping with an external DtN --------------------------------------------
  // rhs_g: the RHS of (eta, psi) with G supplied on the grid; G is projected
  // onto the band by its entry transform, eta_t = P_B G.
  {
    auto &seq = P.rhs_g;
    entry(seq);
    seq.push_back(row_launch(L_ROW_BASE, {entry_g_prog}));
    TaskSpec tg;
    tg.fwd = mbA;
    tg.outs.push_back(B.store(bG, {{-1, 0, 1.0}}));
    seq.push_back(B.col_launch(L_COL_BASE, {tg}));
    std::vector<TaskSpec> ts;
    auto one = [&](OutSpec o) {
      TaskSpec t;
      t.outs.push_back(std::move(o));
      ts.push_back(std::move(t));
    };
    one(B.lift(mE, {{bUE[0], 0, kref}}));
    one(B.lift(mEy, {{bUE[0], SYM_IKY, 1.0}}));
    one(B.lift(mP, {{bUP[0], 0, 1.0}}));
    one(B.lift(mPy, {{bUP[0], SYM_IKY, 1.0}}));
    one(B.lift(mG, {{bG, 0, 1.0}}));
    seq.push_back(B.col_launch(L_COL_PAD, ts));
    seq.push_back(row_launch(L_ROW_PAD, {bern_prog}));
    TaskSpec t = B.fold_task(mN);
    t.outs.push_back(B.store(bPT, {{bUE[0], 0, -g}, {-1, 0, 1.0}}));
    seq.push_back(B.col_launch(L_COL_PAD, {t}));
    exit_seq(seq, bG, bPT);
  }
  // filter: A(k) on (eta, psi) (eq:state_filter), identity when the filter is off
  {
    auto &seq = P.filter;
    entry(seq);
    std::vector<TaskSpec> ts(2);
    ts[0].outs.push_back(B.lift(mbA, {{bUE[0], FILT, 1.0}}));
    ts[1].outs.push_back(B.lift(mbB, {{bUP[0], FILT, 1.0}}));
    seq.push_back(B.col_launch(L_COL_BASE, ts));
    seq.push_back(row_launch(L_ROW_BASE, {exit2_prog}));
  }

  // ---- algorithmic bytes and FFT flops per launch ------------------------------
  // Every program or task streams its fields through HBM once: a row program
  // reads each mixed field it loads (kx < nx/2 of one row per team) and writes
  // each field it stores; a column task reads the mixed field it folds and the
  // base spectra of its terms and writes its stores and lifts.
  {
    const double rb = pp.real_bytes, cb = 2.0 * rb, K = pp.nx / 2;
    const double rows_pad = pp.ny > 1 ? 1.5 * pp.ny : 1.0, rows_base = pp.ny;
    auto fft_flops = [](double n) { return 5.0 * n * std::log2(n); };
    auto annotate = [&](std::vector<Launch> &seq) {
      for (auto &l : seq) {
        l.bytes = l.flops = 0.0;
        if (l.kind == L_ROW_PAD || l.kind == L_ROW_BASE) {
          const double rows = l.kind == L_ROW_PAD ? rows_pad : rows_base;
          const double nrow = l.kind == L_ROW_PAD ? 1.5 * pp.nx : pp.nx;
          for (int k = l.first; k < l.first + l.count; ++k) {
            const RowProg &pg = P.progs[k];
            for (int i = 0; i < pg.nop; ++i) {
              const RowOp &o = P.ops[pg.op0 + i];
              const int nf = (o.fa >= 0) + (o.fb >= 0);
              if (o.code == OP_LD2) {
                l.bytes += nf * rows * K * cb;
                l.flops += rows * fft_flops(nrow);
              } else if (o.code == OP_ST2) {
                l.bytes += nf * rows * K * cb;
                l.flops += rows * fft_flops(nrow);
              } else if (o.code == OP_LDP || o.code == OP_STP) {
                l.bytes += (o.code == OP_LDP ? nf : 1) * rows * pp.nx * 8.0;
              }
            }
          }
        } else if (l.kind == L_COL_PAD || l.kind == L_COL_BASE) {
          const double rows = l.kind == L_COL_PAD ? rows_pad : rows_base;
          for (int k = l.first; k < l.first + l.count; ++k) {
            const ColTask &t = P.tasks[k];
            for (int f = 0; f < kMaxFolds; ++f)
              if (t.fwd[f] >= 0) {
                l.bytes += rows * K * cb;
                l.flops += K * fft_flops(rows);
              }
            for (int i = 0; i < t.no; ++i) {
              const ColOut &o = P.outs[t.o0 + i];
              for (int j = 0; j < o.nt; ++j)
                if (P.terms[o.t0 + j].src >= 0) l.bytes += rows_base * K * 16.0;
              if (o.dst_base >= 0) l.bytes += rows_base * K * 16.0;
              if (o.dst_mixed >= 0) {
                l.bytes += rows * K * cb;
                l.flops += K * fft_flops(rows);
              }
            }
          }
        } else if (l.kind == L_PARSEVAL) {
          l.bytes = 4.0 * rows_base * K * 16.0;
        }
      }
    };
    for (auto *seq : plan_sequences(P)) annotate(*seq);
  }
  return P;
}

std::vector<std::vector<Launch> *> plan_sequences(Plan &p) {
  std::vector<std::vector<Launch> *> v = {&p.dtn,          &p.rhs,          &p.ham,          &p.step_entry,
                                          &p.step_body[0], &p.step_body[1], &p.step_lift[0], &p.step_lift[1],
                                          &p.step_exit[0], &p.step_exit[1], &p.rhs_g,        &p.filter,
                                          &p.ab2_first[0], &p.ab2_first[1], &p.ab2_body[0],  &p.ab2_body[1],
                                          &p.inv_entry,    &p.inv_iter,     &p.inv_exit,     &p.lift_phi};
  for (int r = 1; r <= p.depth_chunk_max; ++r) v.push_back(&p.depth_chunk[r]);
  return v;
}

std::string validate_plan(const Plan &p, int rows_pad, int rows_base) {
  (void)rows_pad;
  (void)rows_base;
  auto bad = [](const std::string &m) { return m; };
  for (auto &pg : p.progs) {
    if (pg.op0 < 0 || pg.nop < 0 || pg.op0 + pg.nop > (int)p.ops.size()) return bad("program range");
    for (int i = 0; i < pg.nop; ++i) {
      const RowOp &o = p.ops[pg.op0 + i];
      switch (o.code) {
        case OP_LD2:
          if (o.fa < 0 || o.fa >= p.nmix || o.fb >= p.nmix) return bad("LD2 field");
          break;
        case OP_ST2:
          if (o.fa < 0 || o.fa >= p.nmix || o.fb >= p.nmix) return bad("ST2 field");
          if (o.a > RS_O2 || (o.b != RS_NONE && o.b > RS_O2)) return bad("ST2 reg");
          if ((o.a == RS_U) != (o.b == RS_V) || o.a == RS_V || o.b == RS_U) return bad("ST2 pairs u with a set");
          break;
        case OP_LDP:
          if (o.fa < 0 || o.fa > 2 || o.fb > 2) return bad("LDP slot");
          break;
        case OP_STP:
          if (o.fa < 0 || o.fa > 1 || o.a > RS_O2 || o.fb >= 3 * kMaxChunkLayers) return bad("STP");
          break;
        case OP_MAC:
          if (o.a < RS_O0 || o.a > RS_O2 || o.b > RS_A || o.c > RS_A) return bad("MAC regs");
          break;
        case OP_MOV:
          if (o.a != RS_A || o.b > RS_A) return bad("MOV regs");
          break;
        case OP_ZERO:
          if (o.a > RS_O2) return bad("ZERO reg");
          break;
        case OP_BERN:
          break;
        default:
          return bad("op code");
      }
    }
  }
  for (auto &t : p.tasks) {
    for (int f = 0; f < kMaxFolds; ++f)
      if (t.fwd[f] >= p.nmix || (f > 0 && t.fwd[f] >= 0 && t.fwd[f - 1] < 0)) return bad("task fwd");
    if (t.o0 < 0 || t.no < 0 || t.o0 + t.no > (int)p.outs.size()) return bad("task outs");
    for (int i = 0; i < t.no; ++i) {
      const ColOut &o = p.outs[t.o0 + i];
      if (o.dst_base >= p.nbase || o.dst_mixed >= p.nmix) return bad("out dst");
      if (o.t0 < 0 || o.nt < 0 || o.t0 + o.nt > (int)p.terms.size()) return bad("out terms");
      for (int k = 0; k < o.nt; ++k) {
        const ColTerm &tm = p.terms[o.t0 + k];
        if (tm.src >= p.nbase) return bad("term src");
        if (tm.src < 0 && t.fwd[0] < 0) return bad("term uses missing fold");
        // the kernels read the taper table only for tasks that fold
        if (tm.sym & SYM_TAPER) return bad("taper on an output term");
      }
    }
  }
  auto chk = [&](const std::vector<Launch> &seq) -> std::string {
    for (auto &l : seq) {
      if (l.kind == L_ROW_PAD || l.kind == L_ROW_BASE) {
        if (l.first < 0 || l.count < 1 || l.first + l.count > (int)p.progs.size()) return "row launch";
        for (int k = l.first; k < l.first + l.count; ++k)
          for (int i = 0; i < p.progs[k].nop; ++i) {
            const int code = p.ops[p.progs[k].op0 + i].code;
            if (l.kind == L_ROW_PAD && (code == OP_LDP || code == OP_STP)) return "caller field op on padded rows";
          }
      } else if (l.kind == L_COL_PAD || l.kind == L_COL_BASE) {
        if (l.first < 0 || l.count < 1 || l.first + l.count > (int)p.tasks.size()) return "col launch";
        if (l.c2 != 0 && !(l.c2 == 1 && l.kind == L_COL_BASE)) return "lift_sym variant on a padded pass";
        if (l.d2 != 0 && !(l.d2 == kMaxFolds && l.c2 == 0)) return "fold teams on a lift_sym launch";
        // one lift per mixed field per launch (blocks of one launch run in any order)
        std::vector<char> lifted(p.nmix, 0);
        for (int k = l.first; k < l.first + l.count; ++k)
          for (int i = 0; i < p.tasks[k].no; ++i) {
            const int d = p.outs[p.tasks[k].o0 + i].dst_mixed;
            if (d >= 0 && lifted[d]++) return "mixed field lifted twice in one launch";
          }
        for (int k = l.first; k < l.first + l.count; ++k)
          for (int i = 0; i < p.tasks[k].no; ++i)
            if (p.outs[p.tasks[k].o0 + i].lift_sym && l.c2 != 1) return "lift_sym output in a plain column launch";
      } else if (l.kind == L_PARSEVAL) {
        if (l.first >= p.nbase || l.count >= p.nbase || l.c2 >= p.nbase || l.d2 >= p.nbase) return "parseval";
      } else {
        return "launch kind";
      }
    }
    return "";
  };
  for (auto *seq : plan_sequences(const_cast<Plan &>(p))) {
    std::string e = chk(*seq);
    if (!e.empty()) return e;
  }
  return "";
}

}  // namespace zk
