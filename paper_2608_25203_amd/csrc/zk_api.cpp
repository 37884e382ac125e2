// zk_api.cpp -- context, workspace layout, schedule upload and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "zk.h"
#include "zk_kernels.hpp"
#include "zk_plan.hpp"
#include "zk_ctx_internal.hpp"

using namespace zk;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }


int fail(zk_ctx *c, int code, const std::string &m) {
  if (c) c->err = m;
  return code;
}
int hip_fail(zk_ctx *c, hipError_t e, const char *what) {
  return fail(c, ZK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIP_TRY(c, call)                          \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(c, e_, #call); \
  } while (0)

size_t real_size(const zk_ctx *c) { return c->precision == 32 ? sizeof(float) : sizeof(double); }

hipError_t take_event(zk_ctx *c, hipEvent_t *e) {
  if (!c->pool.empty()) {
    *e = c->pool.back();
    c->pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Wait for pending launch events and fold them into the per-kind totals.
int flush_prof(zk_ctx *c) {
  if (c->pending.empty()) return ZK_OK;
  HIP_TRY(c, hipEventSynchronize(c->pending.back().b));
  for (auto &r : c->pending) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, r.a, r.b));
    c->st_ms[r.kind] += ms;
    c->st_bytes[r.kind] += r.bytes;
    c->st_flops[r.kind] += r.flops;
    c->st_n[r.kind] += 1;
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->pending.clear();
  return ZK_OK;
}

// Schedule capacities: plans for the same (nx, ny, M) have identical sizes
// for every dt and option, so one capacity computed at layout time suffices.
void compute_layout(zk_ctx *c) {
  const int nx = c->pp.nx, ny = c->pp.ny;
  const size_t rs = real_size(c);
  const size_t cs = 2 * rs;
  const int lens[4] = {3 * nx / 2, nx, 3 * ny / 2, ny};
  size_t off = 0;
  for (int i = 0; i < 4; ++i) {  // kTwSlots twiddle tables per transform length
    c->off_tw[i] = off;
    off = align_up(off + (size_t)kTwSlots * lens[i] * cs);
  }
  Plan probe = build_plan(c->pp, 1.0);
  c->sched_cap[0] = probe.ops.size();
  c->sched_cap[1] = probe.progs.size();
  c->sched_cap[2] = probe.terms.size();
  c->sched_cap[3] = probe.outs.size();
  c->sched_cap[4] = probe.tasks.size();
  c->off_ops = off;
  off = align_up(off + c->sched_cap[0] * sizeof(RowOp));
  c->off_progs = off;
  off = align_up(off + c->sched_cap[1] * sizeof(RowProg));
  c->off_terms = off;
  off = align_up(off + c->sched_cap[2] * sizeof(ColTerm));
  c->off_outs = off;
  off = align_up(off + c->sched_cap[3] * sizeof(ColOut));
  c->off_tasks = off;
  off = align_up(off + c->sched_cap[4] * sizeof(ColTask));
  c->off_rargs = off;  // [pad, base] row argument records
  off = align_up(off + 2 * std::max(sizeof(RowArgs<double>), sizeof(RowArgs<float>)));
  c->off_cargs = off;  // [pad, base] column argument records
  off = align_up(off + 2 * std::max(sizeof(ColArgs<double>), sizeof(ColArgs<float>)));
  c->off_iprog = off;  // items {pad 0 | base 1, program}, pad block then base block
  off = align_up(off + 2 * c->sched_cap[1] * sizeof(BatchItem));
  c->off_itask = off;  // items {pad 0 | base 1, task}
  off = align_up(off + 2 * c->sched_cap[4] * sizeof(BatchItem));
  c->off_ifsym = 0;
  if (c->integrator == ZK_INTEGRATOR_IFAB2) {
    c->off_ifsym = off;
    off = align_up(off + (size_t)(nx / 2) * ny * kIfCoefs * sizeof(double));
  }
  c->off_layer = off;  // depths of one chunk of layers
  off = align_up(off + kMaxChunkLayers * sizeof(double));
  c->off_ext = 0;
  if (c->bc == ZK_BC_REFLECT) {
    c->off_ext = off;
    off = align_up(off + 4 * (size_t)nx * ny * sizeof(double));
  }
  c->off_red = off;
  off = align_up(off + (2 * kRedBlocks + 8) * sizeof(double));
  c->off_cmax = off;
  off = align_up(off + (size_t)probe.nmix * (nx / 2) * sizeof(float));
  c->off_sym = off;
  off = align_up(off + 2 * (size_t)(nx / 2) * ny * sizeof(double));  // G0 table, then the taper table
  c->off_fx = off;
  off = align_up(off + (size_t)(nx / 2) * sizeof(double));
  c->off_fy = off;
  off = align_up(off + (size_t)ny * sizeof(double));
  c->base_stride = (long long)(align_up((size_t)(nx / 2) * ny * 16) / 16);
  c->off_base = off;
  off = align_up(off + (size_t)probe.nbase * c->base_stride * 16);
  c->mix_stride = (long long)(align_up((size_t)(nx / 2) * (3 * ny / 2) * cs) / cs);
  c->off_mix = off;
  off = align_up(off + (size_t)probe.nmix * c->mix_stride * cs);
  c->total = off;
}

// The kTwSlots twiddle tables of transform length n: one pass-ordered table
// per first-pass radix E of slot tw_slot(E) (see stage order in zk_fft.hpp):
// entry Ns_p - E + (r-1) Ns_p + k of table E is W_n^(r k step_p); a slot
// whose E does not give a valid team is unused; and the natural table W_n^m,
// m < n, in slot kTwNatural.  In long double on the host.
template <typename real>
std::vector<cpx<real>> twiddles(int n) {
  std::vector<cpx<real>> t((size_t)kTwSlots * n, cpx<real>{(real)0, (real)0});
  const long double two_pi = 2.0L * 3.14159265358979323846264338327950288L;
  for (int m = 0; m < n; ++m) {
    const long double a = -two_pi * (long double)m / (long double)n;
    t[(size_t)kTwNatural * n + m] = {(real)cosl(a), (real)sinl(a)};
  }
  // candidate first-pass radices of this length, one per slot (tw_slot)
  const bool f5 = n % 5 == 0;  // 5 2^k lengths: one candidate, 15 (padded) or 10 (base)
  const int cand[kTwNatural] = {f5 ? (n % 3 == 0 ? 15 : 10) : (n % 9 == 0 ? 9 : (n % 3 == 0 ? 3 : 2)),
                                f5 ? 0 : (n % 9 == 0 ? 18 : (n % 3 == 0 ? 6 : 4)),
                                f5 || n % 9 == 0 ? 0 : (n % 3 == 0 ? 12 : 8)};
  for (int s = 0; s < kTwNatural; ++s) {
    const int E = cand[s];
    if (E == 0) continue;
    const int T = n / E;
    if (n % E || T < 2 || (T & (T - 1)) || num_passes(T, E) < 2) continue;
    cpx<real> *tab = t.data() + (size_t)s * n;
    int ns = E;
    for (int p = 1; p < num_passes(T, E); ++p) {
      const int rp = later_radix(T, E, p), step = n / (ns * rp);
      for (int r = 1; r < rp; ++r)
        for (int k = 0; k < ns; ++k) {
          const long double a = -two_pi * (long double)(r * k * step) / (long double)n;
          tab[ns - E + (r - 1) * ns + k] = {(real)cosl(a), (real)sinl(a)};
        }
      ns *= rp;
    }
  }
  return t;
}

// The compiled shape (zk_row_shapes.hpp) whose op sequence a program's ops
// match in (code, a, b, c), or -1.
static int row_shape_of(const RowOp *ops, int nop) {
  for (int sh = 0; sh < kRowShapes; ++sh) {
    if (kRowShapeLen[sh] != nop) continue;
    bool same = true;
    for (int i = 0; i < nop && same; ++i) {
      const RowOp &o = ops[i];
      same = kRowShapeOps[sh][i] == ((uint32_t)o.code | (uint32_t)o.a << 8 | (uint32_t)o.b << 16 | (uint32_t)o.c << 24);
    }
    if (same) return sh;
  }
  return -1;
}

int upload(zk_ctx *c, double dt) {
  if (!c->bound) return fail(c, ZK_ENOWS, "workspace not bound");
  const bool need = !c->have_plan || c->dirty || !(dt == c->plan_dt || (std::isnan(dt) && std::isnan(c->plan_dt)));
  if (!need) return ZK_OK;
  try {
    c->plan = build_plan(c->pp, std::isnan(dt) ? 1.0 : dt);
  } catch (const std::exception &e) {
    return fail(c, ZK_EINVAL, std::string("plan: ") + e.what());
  }
  const std::string v = validate_plan(c->plan, 3 * c->pp.ny / 2, c->pp.ny);
  if (!v.empty()) return fail(c, ZK_EINVAL, "plan validation: " + v);
  const Plan &p = c->plan;
  if (p.ops.size() > c->sched_cap[0] || p.progs.size() > c->sched_cap[1] || p.terms.size() > c->sched_cap[2] ||
      p.outs.size() > c->sched_cap[3] || p.tasks.size() > c->sched_cap[4])
    return fail(c, ZK_EINVAL, "schedule exceeds reserved capacity");
  HIP_TRY(c, hipSetDevice(c->device));
  auto put = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
    if (!bytes) return hipSuccess;
    return hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->stream);
  };
  HIP_TRY(c, put(c->off_ops, p.ops.data(), p.ops.size() * sizeof(RowOp)));
  // Tag each program with its compiled shape (kernels without compiled
  // shapes, and untagged programs, interpret the op list).
  std::vector<RowProg> progs = p.progs;
  if (c->row_programs)
    for (RowProg &pg : progs) pg.shape1 = 1 + row_shape_of(p.ops.data() + pg.op0, pg.nop);
  HIP_TRY(c, put(c->off_progs, progs.data(), progs.size() * sizeof(RowProg)));
  HIP_TRY(c, put(c->off_terms, p.terms.data(), p.terms.size() * sizeof(ColTerm)));
  HIP_TRY(c, put(c->off_outs, p.outs.data(), p.outs.size() * sizeof(ColOut)));
  HIP_TRY(c, put(c->off_tasks, p.tasks.data(), p.tasks.size() * sizeof(ColTask)));
  if (c->dirty) {
    const int nx = c->pp.nx, ny = c->pp.ny;
    // Fourier symbol tables (long double on the host, stored as FP64):
    // G0 = |k| tanh(|k| d) and the taper exp(-(|k|/kc)^8) per band element in
    // the tiled base-spectrum layout; separable filter factors per axis.
    {
      const long double pi = 3.14159265358979323846264338327950288L;
      const long double kxs = 2 * pi / c->pp.Lx, kys = 2 * pi / c->pp.Ly;
      // kNyq over the axes that have one (a 1D grid, ny = 1, has only x)
      const long double kc =
          2.0L / 3.0L * (ny > 1 ? std::min(pi * nx / c->pp.Lx, pi * ny / c->pp.Ly) : pi * nx / c->pp.Lx);
      const size_t nel = (size_t)(nx / 2) * ny;
      std::vector<double> tab(2 * nel);  // [G0 | taper]
      for (int col = 0; col < nx / 2; ++col)
        for (int b = 0; b < ny; ++b) {
          const int my = (b < ny / 2 || ny == 1) ? b : b - ny;  // a 1D grid's one row is ky = 0
          const long double kx = kxs * col, ky = kys * my;
          const long double kk = sqrtl(kx * kx + ky * ky);
          const long double r = kk / kc, r2 = r * r, r4 = r2 * r2;
          const size_t e = ((size_t)(col / CBB) * ny + b) * CBB + col % CBB;
          tab[e] = (double)(c->pp.depth > 0 ? kk * tanhl(kk * c->pp.depth) : kk);
          tab[nel + e] = (double)expl(-(r4 * r4));
        }
      auto f1 = [&](int m, int n) {
        const long double th = 2 * pi * m / n;
        return (double)((5 + 4 * cosl(th) - cosl(2 * th)) / 8);
      };
      std::vector<double> fx(nx / 2), fy(ny);
      for (int col = 0; col < nx / 2; ++col) fx[col] = f1(col, nx);
      for (int b = 0; b < ny; ++b) fy[b] = f1((b < ny / 2 || ny == 1) ? b : b - ny, ny);
      HIP_TRY(c, put(c->off_sym, tab.data(), tab.size() * sizeof(double)));
      HIP_TRY(c, put(c->off_fx, fx.data(), fx.size() * sizeof(double)));
      HIP_TRY(c, put(c->off_fy, fy.data(), fy.size() * sizeof(double)));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    const int lens[4] = {3 * nx / 2, nx, 3 * ny / 2, ny};
    for (int i = 0; i < 4; ++i) {
      if (c->precision == 32) {
        auto t = twiddles<float>(lens[i]);
        HIP_TRY(c, put(c->off_tw[i], t.data(), t.size() * sizeof(t[0])));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
      } else {
        auto t = twiddles<double>(lens[i]);
        HIP_TRY(c, put(c->off_tw[i], t.data(), t.size() * sizeof(t[0])));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
      }
    }
  }
  {
    // argument records (field pointers come with each call) and items
    std::vector<char> rt(2 * std::max(sizeof(RowArgs<double>), sizeof(RowArgs<float>)));
    std::vector<char> ct(2 * std::max(sizeof(ColArgs<double>), sizeof(ColArgs<float>)));
    const Phys none;
    for (int p = 0; p < 2; ++p) {
      if (c->precision == 32) {
        const RowArgs<float> r = ctx_row_args<float>(c, p == 0, none, 0);
        const ColArgs<float> k = ctx_col_args<float>(c, p == 0, 0);
        std::memcpy(&rt[p * sizeof(r)], &r, sizeof(r));
        std::memcpy(&ct[p * sizeof(k)], &k, sizeof(k));
      } else {
        const RowArgs<double> r = ctx_row_args<double>(c, p == 0, none, 0);
        const ColArgs<double> k = ctx_col_args<double>(c, p == 0, 0);
        std::memcpy(&rt[p * sizeof(r)], &r, sizeof(r));
        std::memcpy(&ct[p * sizeof(k)], &k, sizeof(k));
      }
    }
    std::vector<BatchItem> ip(2 * c->sched_cap[1]), it(2 * c->sched_cap[4]);
    for (size_t k = 0; k < c->sched_cap[1]; ++k) {
      ip[k] = BatchItem{0, (int32_t)k};
      ip[c->sched_cap[1] + k] = BatchItem{1, (int32_t)k};
    }
    for (size_t k = 0; k < c->sched_cap[4]; ++k) {
      it[k] = BatchItem{0, (int32_t)k};
      it[c->sched_cap[4] + k] = BatchItem{1, (int32_t)k};
    }
    HIP_TRY(c, put(c->off_rargs, rt.data(), rt.size()));
    HIP_TRY(c, put(c->off_cargs, ct.data(), ct.size()));
    HIP_TRY(c, put(c->off_iprog, ip.data(), ip.size() * sizeof(BatchItem)));
    HIP_TRY(c, put(c->off_itask, it.data(), it.size() * sizeof(BatchItem)));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  if (c->integrator == ZK_INTEGRATOR_IFAB2 && !std::isnan(dt) && (c->dirty || !(dt == c->ifsym_dt))) {
    // exact linear flow and its constant-forcing response over dt per band
    // element (Sec. 3.4), omega^2 = g G0, in long double; k = 0 limits
    const int nx = c->pp.nx, ny = c->pp.ny;
    const long double pi = 3.14159265358979323846264338327950288L;
    const long double kxs = 2 * pi / c->pp.Lx, kys = 2 * pi / c->pp.Ly, g = c->pp.g, h = dt;
    std::vector<double> tab((size_t)(nx / 2) * ny * kIfCoefs);
    for (int col = 0; col < nx / 2; ++col)
      for (int b = 0; b < ny; ++b) {
        const int my = (b < ny / 2 || ny == 1) ? b : b - ny;
        const long double kx = kxs * col, ky = kys * my, kk = sqrtl(kx * kx + ky * ky);
        const long double G0 = c->pp.depth > 0 ? kk * tanhl(kk * c->pp.depth) : kk;
        const long double om = sqrtl(g * G0);
        long double v[kIfCoefs];
        if (om == 0) {
          v[0] = 1;
          v[1] = 0;
          v[2] = g * h;
          v[3] = h;
          v[4] = 0;
          v[5] = 0.5L * g * h * h;
        } else {
          const long double cs = cosl(om * h), sn = sinl(om * h);
          v[0] = cs;
          v[1] = G0 * sn / om;
          v[2] = g * sn / om;
          v[3] = sn / om;
          v[4] = (1 - cs) / g;
          v[5] = (1 - cs) / G0;
        }
        const size_t e = ((size_t)(col / CBB) * ny + b) * CBB + col % CBB;
        for (int k = 0; k < kIfCoefs; ++k) tab[e * kIfCoefs + k] = (double)v[k];
      }
    HIP_TRY(c, put(c->off_ifsym, tab.data(), tab.size() * sizeof(double)));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->ifsym_dt = dt;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // host vectors may change after return
  c->plan_dt = dt;
  c->have_plan = true;
  c->dirty = false;
  return ZK_OK;
}

template <typename real>
int run_seq_t(zk_ctx *c, const std::vector<Launch> &seq, const Phys &ph) {
  const int nx = c->pp.nx, ny = c->pp.ny;
  char *ws = c->ws;
  cpx<double> *base = reinterpret_cast<cpx<double> *>(ws + c->off_base);
  for (const Launch &l : seq) {
    hipError_t e = hipSuccess;
    zk_ctx::Rec rec{l.kind, l.bytes, l.flops, nullptr, nullptr};
    if (c->prof) {
      HIP_TRY(c, take_event(c, &rec.a));
      HIP_TRY(c, take_event(c, &rec.b));
      HIP_TRY(c, hipEventRecord(rec.a, c->stream));
    }
    if (l.kind != L_PARSEVAL) {
      const bool row = l.kind == L_ROW_PAD || l.kind == L_ROW_BASE;
      const bool pad = l.kind == L_ROW_PAD || l.kind == L_COL_PAD;
      const TeamShape sh = ctx_team(c, row, pad);
      // a single grid passes no item table: block row y runs program or task
      // l.first + y of argument record 0 (padded passes) or 1 (base passes),
      // from the program or task table passed with the launch
      const BatchItem *items = nullptr;
      const int tile0 = pad ? 0 : 1, first0 = l.first;
      const void *sched0 = ws + (row ? c->off_progs : c->off_tasks);
      const PhysArgs pa{ph.in0, ph.in1, ph.in2, ph.out0, ph.out1, 1};
      const dim3 grid(sh.blocks, l.count);
      const ColArgs<real> *cargs = reinterpret_cast<const ColArgs<real> *>(ws + c->off_cargs);
      if (!row && c->pp.ny == 1)  // 1D grid: one element per column, no y transform
        e = launch_col_1d<real>(l.c2 == 1, dim3((nx / 2 + 255) / 256, l.count), c->stream, cargs, tile0, first0);
      else if (row && pad && c->row_fft == ZK_ROW_FFT_LANES && row_lanes_ok(sh.T, sh.E, true, (int)sizeof(real)))
        e = launch_lanes_row<real>(sh.T, sh.E, grid, c->stream,
                                   reinterpret_cast<const RowArgs<real> *>(ws + c->off_rargs), items, tile0, first0,
                                   sched0, pa);
      else if (row)
        e = launch_batch_row<real>(sh.T, sh.E, pad, grid, c->stream,
                                   reinterpret_cast<const RowArgs<real> *>(ws + c->off_rargs), items, tile0, first0,
                                   sched0, pa);
      else if (l.c2 == 1)
        e = launch_batch_col_lift<real>(sh.T, sh.E, grid, c->stream, cargs, items, tile0, first0, sched0, pa);
      else if (l.d2 == kMaxFolds && fold_team_shape(sh.T, sh.E))  // one block per column
        e = launch_batch_col_folds<real>(sh.T, sh.E, dim3(nx / 2, l.count), c->stream, cargs, items, tile0, first0,
                                         sched0, pa);
      else
        e = launch_batch_col<real>(sh.T, sh.E, pad, grid, c->stream, cargs, items, tile0, first0, sched0, pa);
    } else {
      double *red = reinterpret_cast<double *>(ws + c->off_red);
      e = launch_parseval(base + (long long)l.first * c->base_stride, base + (long long)l.count * c->base_stride,
                          base + (long long)l.c2 * c->base_stride, base + (long long)l.d2 * c->base_stride, nx / 2, ny,
                          red, red + 2 * kRedBlocks, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
    if (c->prof) {
      HIP_TRY(c, hipEventRecord(rec.b, c->stream));
      c->pending.push_back(rec);
      if (c->pending.size() >= 4096) {
        const int rc = flush_prof(c);
        if (rc) return rc;
      }
    }
  }
  return ZK_OK;
}

int run_seq(zk_ctx *c, const std::vector<Launch> &seq, const Phys &ph) {
  return c->precision == 32 ? run_seq_t<float>(c, seq, ph) : run_seq_t<double>(c, seq, ph);
}

int check_call(zk_ctx *c) {
  if (!c) return ZK_EINVAL;
  c->err.clear();
  if (!c->bound) return fail(c, ZK_ENOWS, "workspace not bound (call zk_bind)");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  return ZK_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Reflecting walls: the caller's fields are mirrored into doubled workspace
// fields ext(k) before a sequence and its outputs cropped back after.
double *ext(zk_ctx *c, int k) {
  return reinterpret_cast<double *>(c->ws + c->off_ext) + (size_t)k * c->pp.nx * c->pp.ny;
}
int mirror_in(zk_ctx *c, const double *a, int k) {
  HIP_TRY(c, launch_mirror(a, c->unx, c->uny, ext(c, k), c->stream));
  return ZK_OK;
}
int crop_out(zk_ctx *c, int k, double *a) {
  HIP_TRY(c, launch_crop(ext(c, k), c->unx, c->uny, a, c->stream));
  return ZK_OK;
}

}  // namespace

namespace zk {

TeamShape ctx_team(const zk_ctx *c, bool row, bool pad) {
  // default: the smallest first-pass radix (E = 3 padded, 2 base), i.e.
  // T = N / E threads per transform (at most 1024 for n <= 2048), or the
  // autotuned shape; a block has max(256, T) threads, 256 / T teams when T < 256
  const int n = row ? c->pp.nx : c->pp.ny;
  const int N = pad ? 3 * n / 2 : n;
  TeamShape sh;
  if (!row && n == 1) {  // a 1D grid's columns: one thread per column (col_kernel_1d)
    sh.T = 1;
    sh.E = 1;
    sh.blocks = (c->pp.nx / 2 + 255) / 256;
    return sh;
  }
  sh.T = c->tuneT[row][pad] ? c->tuneT[row][pad] : N / default_radix(n, pad);
  sh.E = N / sh.T;
  const int tpb = sh.T < 256 ? 256 / sh.T : 1;
  // (rows of a 1D grid: 1, in a block whose other teams idle)
  sh.blocks = row ? ((pad ? 3 * c->pp.ny / 2 : c->pp.ny) + tpb - 1) / tpb : (c->pp.nx / 2 + tpb - 1) / tpb;
  return sh;
}

template <typename real>
RowArgs<real> ctx_row_args(const zk_ctx *c, bool pad, const Phys &ph, int prog0) {
  char *ws = c->ws;
  RowArgs<real> a{};
  a.ops = reinterpret_cast<const RowOp *>(ws + c->off_ops);
  a.progs = reinterpret_cast<const RowProg *>(ws + c->off_progs);
  a.prog0 = prog0;
  a.mix = reinterpret_cast<cpx<real> *>(ws + c->off_mix);
  a.mix_stride = c->mix_stride;
  a.rows = pad ? 3 * c->pp.ny / 2 : c->pp.ny;
  a.nx = c->pp.nx;
  a.pin0 = ph.in0;
  a.pin1 = ph.in1;
  a.pin2 = ph.in2;
  a.pout0 = ph.out0;
  a.pout1 = ph.out1;
  a.tw = reinterpret_cast<const cpx<real> *>(ws + c->off_tw[pad ? 0 : 1]);
  a.kx_scale = 2.0 * M_PI / c->pp.Lx;
  a.colmax = reinterpret_cast<const float *>(ws + c->off_cmax);
  return a;
}

template <typename real>
ColArgs<real> ctx_col_args(const zk_ctx *c, bool pad, int task0) {
  char *ws = c->ws;
  const int nx = c->pp.nx, ny = c->pp.ny;
  const double kc = 2.0 / 3.0 * (ny > 1 ? std::min(M_PI * nx / c->pp.Lx, M_PI * ny / c->pp.Ly) : M_PI * nx / c->pp.Lx);
  ColArgs<real> a{};
  a.tasks = reinterpret_cast<const ColTask *>(ws + c->off_tasks);
  a.task0 = task0;
  a.outs = reinterpret_cast<const ColOut *>(ws + c->off_outs);
  a.terms = reinterpret_cast<const ColTerm *>(ws + c->off_terms);
  a.mix = reinterpret_cast<cpx<real> *>(ws + c->off_mix);
  a.mix_stride = c->mix_stride;
  a.rows = pad ? 3 * ny / 2 : ny;
  a.base = reinterpret_cast<cpx<double> *>(ws + c->off_base);
  a.base_stride = c->base_stride;
  a.ny = ny;
  a.nx = nx;
  a.tw = reinterpret_cast<const cpx<real> *>(ws + c->off_tw[pad ? 2 : 3]);
  a.kx_scale = 2.0 * M_PI / c->pp.Lx;
  a.ky_scale = 2.0 * M_PI / c->pp.Ly;
  a.depth = c->pp.depth;
  a.inv_kc = 1.0 / kc;
  a.taper_on = c->pp.taper ? 1 : 0;
  a.colmax = reinterpret_cast<float *>(ws + c->off_cmax);
  a.sym_g0 = reinterpret_cast<const double *>(ws + c->off_sym);
  a.sym_tp = a.sym_g0 + (size_t)(c->pp.nx / 2) * c->pp.ny;
  a.filt_x = reinterpret_cast<const double *>(ws + c->off_fx);
  a.filt_y = reinterpret_cast<const double *>(ws + c->off_fy);
  a.ifsym = c->off_ifsym ? reinterpret_cast<const double *>(ws + c->off_ifsym) : nullptr;
  a.layer_y = reinterpret_cast<const double *>(ws + c->off_layer);
  return a;
}

template RowArgs<double> ctx_row_args<double>(const zk_ctx *, bool, const Phys &, int);
template RowArgs<float> ctx_row_args<float>(const zk_ctx *, bool, const Phys &, int);
template ColArgs<double> ctx_col_args<double>(const zk_ctx *, bool, int);
template ColArgs<float> ctx_col_args<float>(const zk_ctx *, bool, int);

int ctx_upload(zk_ctx *c, double dt) { return upload(c, dt); }

int ctx_prepare(zk_ctx *c) {
  int rc = check_call(c);
  if (rc) return rc;
  return upload(c, c->have_plan ? c->plan_dt : NAN);
}

int ctx_run(zk_ctx *c, const std::vector<Launch> &seq, const Phys &ph) { return run_seq(c, seq, ph); }

}  // namespace zk

extern "C" {

zk_ctx *zk_create(int nx, int ny, double Lx, double Ly, double depth, double g, int M) {
  // ny = 1: a 1D grid.  nx / 2 columns must fill the mixed fields' tiles of
  // 64-byte column groups (8 FP32 or 4 FP64 columns): nx % 16 == 0.
  if (!axis_len_ok(nx) || nx % 16 != 0 || !(axis_len_ok(ny) || ny == 1)) return nullptr;
  if (!(Lx > 0) || !(Ly > 0) || !(g > 0) || M < 1 || M > 8) return nullptr;
  zk_ctx *c = new (std::nothrow) zk_ctx();
  if (!c) return nullptr;
  c->pp.nx = nx;
  c->pp.ny = ny;
  c->pp.Lx = Lx;
  c->pp.Ly = Ly;
  c->pp.depth = (std::isfinite(depth) && depth > 0) ? depth : 0.0;
  c->pp.g = g;
  c->pp.M = M;
  c->pp.eps = 1.0;
  c->pp.taper = true;
  c->pp.filt = true;
  c->pp.real_bytes = 8;
  c->unx = nx;
  c->uny = ny;
  c->uLx = Lx;
  c->uLy = Ly;
  try {
    compute_layout(c);
  } catch (...) {
    delete c;
    return nullptr;
  }
  return c;
}

void zk_destroy(zk_ctx *c) { delete c; }

int zk_set_option(zk_ctx *c, int key, double v) {
  if (!c) return ZK_EINVAL;
  c->err.clear();
  switch (key) {
    case ZK_OPT_EPS:
      if (!(v >= 0.0 && v <= 1.0)) return fail(c, ZK_EINVAL, "eps must be in [0, 1]");
      c->pp.eps = v;
      break;
    case ZK_OPT_TAPER:
      c->pp.taper = v != 0.0;
      break;
    case ZK_OPT_FILTER:
      c->pp.filt = v != 0.0;
      break;
    case ZK_OPT_PRECISION:
      if (v != 32.0 && v != 64.0) return fail(c, ZK_EINVAL, "precision must be 32 or 64");
      if (c->bound && (int)v != c->precision) return fail(c, ZK_EINVAL, "set precision before zk_bind");
      c->precision = (int)v;
      c->pp.real_bytes = c->precision == 32 ? 4 : 8;
      compute_layout(c);
      break;
    case ZK_OPT_CHECK:
      c->check = v != 0.0;
      return ZK_OK;
    case ZK_OPT_PROFILE:
      c->prof = v != 0.0;
      return ZK_OK;
    case ZK_OPT_ROW_FFT:
      if (v != ZK_ROW_FFT_STOCKHAM && v != ZK_ROW_FFT_LANES) return fail(c, ZK_EINVAL, "unknown row transform form");
      c->row_fft = (int)v;
      return ZK_OK;
    case ZK_OPT_ROW_PROGRAMS:
      if (v != 0.0 && v != 1.0) return fail(c, ZK_EINVAL, "row programs option must be 0 or 1");
      c->row_programs = (int)v;
      c->dirty = true;  // re-tag the uploaded programs; the plan itself is unchanged
      return ZK_OK;
    case ZK_OPT_BOUNDARY:
      if (v != ZK_BC_PERIODIC && v != ZK_BC_REFLECT) return fail(c, ZK_EINVAL, "unknown boundary");
      if (c->bound && (int)v != c->bc) return fail(c, ZK_EINVAL, "set the boundary before zk_bind");
      if (v == ZK_BC_REFLECT && (!axis_len_ok(2 * c->unx) || !axis_len_ok(2 * c->uny)))
        return fail(c, ZK_EINVAL, "reflecting walls double the grid: 2 nx and 2 ny must be built lengths");
      c->bc = (int)v;
      c->pp.nx = c->bc ? 2 * c->unx : c->unx;
      c->pp.ny = c->bc ? 2 * c->uny : c->uny;
      c->pp.Lx = c->bc ? 2 * c->uLx : c->uLx;
      c->pp.Ly = c->bc ? 2 * c->uLy : c->uLy;
      compute_layout(c);
      break;
    case ZK_OPT_INTEGRATOR:
      if (v != ZK_INTEGRATOR_RK4 && v != ZK_INTEGRATOR_IFAB2) return fail(c, ZK_EINVAL, "unknown integrator");
      if (c->bound && (int)v != c->integrator) return fail(c, ZK_EINVAL, "set the integrator before zk_bind");
      c->integrator = (int)v;
      compute_layout(c);
      break;
    default:
      return fail(c, ZK_EINVAL, "unknown option");
  }
  c->dirty = true;
  c->have_plan = false;
  return ZK_OK;
}

int zk_get_option(const zk_ctx *c, int key, double *v) {
  if (!c || !v) return ZK_EINVAL;
  switch (key) {
    case ZK_OPT_EPS: *v = c->pp.eps; break;
    case ZK_OPT_TAPER: *v = c->pp.taper ? 1.0 : 0.0; break;
    case ZK_OPT_FILTER: *v = c->pp.filt ? 1.0 : 0.0; break;
    case ZK_OPT_PRECISION: *v = c->precision; break;
    case ZK_OPT_CHECK: *v = c->check ? 1.0 : 0.0; break;
    case ZK_OPT_PROFILE: *v = c->prof ? 1.0 : 0.0; break;
    case ZK_OPT_INTEGRATOR: *v = c->integrator; break;
    case ZK_OPT_BOUNDARY: *v = c->bc; break;
    case ZK_OPT_ROW_PROGRAMS: *v = c->row_programs; break;
    case ZK_OPT_ROW_FFT: {  // the form the padded row passes run in at the current team shape
      const TeamShape sh = ctx_team(c, true, true);
      *v = c->row_fft == ZK_ROW_FFT_LANES && row_lanes_ok(sh.T, sh.E, true, c->precision == 32 ? 4 : 8)
               ? ZK_ROW_FFT_LANES
               : ZK_ROW_FFT_STOCKHAM;
      break;
    }
    default: return ZK_EINVAL;
  }
  return ZK_OK;
}

size_t zk_workspace_bytes(const zk_ctx *c) { return c ? c->total : 0; }

int zk_bind(zk_ctx *c, void *ws, size_t bytes, void *stream) {
  if (!c) return ZK_EINVAL;
  c->err.clear();
  if (!ws || ((uintptr_t)ws % kAlign) != 0) return fail(c, ZK_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < c->total) return fail(c, ZK_ENOWS, "workspace smaller than zk_workspace_bytes");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
  c->ws = static_cast<char *>(ws);
  c->ws_bytes = bytes;
  c->stream = static_cast<hipStream_t>(stream);
  c->device = dev;
  c->bound = true;
  c->dirty = true;
  c->have_plan = false;
  return upload(c, NAN);
}

int zk_dtn(zk_ctx *c, const double *eta, const double *psi, double *G) {
  int rc = check_call(c);
  if (rc) return rc;
  if (!eta || !psi || !G || !aligned16(eta) || !aligned16(psi) || !aligned16(G))
    return fail(c, ZK_EINVAL, "null or misaligned field pointer");
  if ((rc = upload(c, c->have_plan ? c->plan_dt : NAN))) return rc;
  Phys ph;
  if (c->bc) {
    if ((rc = mirror_in(c, eta, 0)) || (rc = mirror_in(c, psi, 1))) return rc;
    ph.in0 = ext(c, 0);
    ph.in1 = ext(c, 1);
    ph.out0 = ext(c, 2);
    if ((rc = run_seq(c, c->plan.dtn, ph))) return rc;
    return crop_out(c, 2, G);
  }
  ph.in0 = eta;
  ph.in1 = psi;
  ph.out0 = G;
  return run_seq(c, c->plan.dtn, ph);
}

int zk_rhs(zk_ctx *c, const double *eta, const double *psi, double *eta_t, double *psi_t) {
  int rc = check_call(c);
  if (rc) return rc;
  if (!eta || !psi || !eta_t || !psi_t || !aligned16(eta) || !aligned16(psi) || !aligned16(eta_t) ||
      !aligned16(psi_t))
    return fail(c, ZK_EINVAL, "null or misaligned field pointer");
  if ((rc = upload(c, c->have_plan ? c->plan_dt : NAN))) return rc;
  Phys ph;
  if (c->bc) {
    if ((rc = mirror_in(c, eta, 0)) || (rc = mirror_in(c, psi, 1))) return rc;
    ph.in0 = ext(c, 0);
    ph.in1 = ext(c, 1);
    ph.out0 = ext(c, 2);
    ph.out1 = ext(c, 3);
    if ((rc = run_seq(c, c->plan.rhs, ph))) return rc;
    if ((rc = crop_out(c, 2, eta_t))) return rc;
    return crop_out(c, 3, psi_t);
  }
  ph.in0 = eta;
  ph.in1 = psi;
  ph.out0 = eta_t;
  ph.out1 = psi_t;
  return run_seq(c, c->plan.rhs, ph);
}

int zk_step(zk_ctx *c, double *eta, double *psi, double dt, int nsteps) {
  int rc = check_call(c);
  if (rc) return rc;
  if (!eta || !psi || !aligned16(eta) || !aligned16(psi)) return fail(c, ZK_EINVAL, "null or misaligned field pointer");
  if (!(std::isfinite(dt)) || nsteps < 0) return fail(c, ZK_EINVAL, "dt must be finite and nsteps >= 0");
  if (nsteps == 0) return ZK_OK;
  if ((rc = upload(c, dt))) return rc;
  Phys ph;
  ph.in0 = eta;
  ph.in1 = psi;
  ph.out0 = eta;
  ph.out1 = psi;
  if (c->bc) {
    if ((rc = mirror_in(c, eta, 0)) || (rc = mirror_in(c, psi, 1))) return rc;
    ph.in0 = ph.out0 = ext(c, 0);
    ph.in1 = ph.out1 = ext(c, 1);
  }
  const Plan &p = c->plan;
  if ((rc = run_seq(c, p.step_entry, ph))) return rc;
  const bool ab2 = c->integrator == ZK_INTEGRATOR_IFAB2;
  for (int i = 0; i < nsteps; ++i) {
    const int par = i & 1;
    const std::vector<Launch> &body = ab2 ? (i == 0 ? p.ab2_first[par] : p.ab2_body[par]) : p.step_body[par];
    if ((rc = run_seq(c, body, ph))) return rc;
    if (i + 1 < nsteps && (rc = run_seq(c, p.step_lift[1 - par], ph))) return rc;
  }
  const int fin = nsteps & 1;
  if ((rc = run_seq(c, p.step_exit[fin], ph))) return rc;
  if (c->bc && ((rc = crop_out(c, 0, eta)) || (rc = crop_out(c, 1, psi)))) return rc;
  if (c->check) {
    std::vector<Launch> chk{Launch{L_PARSEVAL, p.chk_e[fin], p.chk_e[fin], p.chk_p[fin], p.chk_p[fin], 0.0, 0.0}};
    if ((rc = run_seq(c, chk, ph))) return rc;
    double h[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(h, c->ws + c->off_red + 2 * kRedBlocks * sizeof(double), sizeof(h),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return fail(c, ZK_EDIVERGED, "state is not finite");
  }
  return ZK_OK;
}

int zk_hamiltonian(zk_ctx *c, const double *eta, const double *psi, double *H) {
  int rc = check_call(c);
  if (rc) return rc;
  if (!eta || !psi || !H || !aligned16(eta) || !aligned16(psi)) return fail(c, ZK_EINVAL, "null or misaligned pointer");
  if ((rc = upload(c, c->have_plan ? c->plan_dt : NAN))) return rc;
  Phys ph;
  ph.in0 = eta;
  ph.in1 = psi;
  if (c->bc) {
    if ((rc = mirror_in(c, eta, 0)) || (rc = mirror_in(c, psi, 1))) return rc;
    ph.in0 = ext(c, 0);
    ph.in1 = ext(c, 1);
  }
  if ((rc = run_seq(c, c->plan.ham, ph))) return rc;
  double h[2] = {0, 0};
  HIP_TRY(c, hipMemcpyAsync(h, c->ws + c->off_red + 2 * kRedBlocks * sizeof(double), sizeof(h),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const double N = (double)c->pp.nx * c->pp.ny;
  const double dA = c->pp.Lx * c->pp.Ly / N;
  *H = 0.5 * dA * h[0] / N + 0.5 * c->pp.g * dA * h[1] / N;
  if (c->bc) *H *= 0.25;  // the tank is a quarter of the doubled domain
  return ZK_OK;
}

int zk_kernel_stats(zk_ctx *c, int kind, double *ms, double *bytes, double *flops, long long *launches) {
  if (!c) return ZK_EINVAL;
  c->err.clear();
  if (c->bound) {
    const int rc = flush_prof(c);
    if (rc) return rc;
  }
  if (kind == -1) {
    for (int k = 0; k < 5; ++k) {
      c->st_ms[k] = c->st_bytes[k] = c->st_flops[k] = 0.0;
      c->st_n[k] = 0;
    }
    return ZK_OK;
  }
  if (kind < 0 || kind > 4 || !ms || !bytes || !flops || !launches) return fail(c, ZK_EINVAL, "bad kind or output");
  *ms = c->st_ms[kind];
  *bytes = c->st_bytes[kind];
  *flops = c->st_flops[kind];
  *launches = c->st_n[kind];
  return ZK_OK;
}

int zk_inverse_dtn(zk_ctx *c, const double *eta, const double *v, double *psi, int iters) {
  int rc = check_call(c);
  if (rc) return rc;
  if (!eta || !v || !psi || !aligned16(eta) || !aligned16(v) || !aligned16(psi))
    return fail(c, ZK_EINVAL, "null or misaligned field pointer");
  if (iters < 0 || iters > 1000) return fail(c, ZK_EINVAL, "iters must be in [0, 1000]");
  if ((rc = upload(c, c->have_plan ? c->plan_dt : NAN))) return rc;
  Phys ph;
  ph.in0 = eta;
  ph.in1 = v;
  ph.out0 = psi;
  if (c->bc) {
    if ((rc = mirror_in(c, eta, 0)) || (rc = mirror_in(c, v, 1))) return rc;
    ph.in0 = ext(c, 0);
    ph.in1 = ext(c, 1);
    ph.out0 = ext(c, 2);
  }
  if ((rc = run_seq(c, c->plan.inv_entry, ph))) return rc;
  for (int i = 0; i < iters; ++i)
    if ((rc = run_seq(c, c->plan.inv_iter, ph))) return rc;
  if ((rc = run_seq(c, c->plan.inv_exit, ph))) return rc;
  return c->bc ? crop_out(c, 2, psi) : ZK_OK;
}

int zk_depth_velocity(zk_ctx *c, const double *eta, const double *psi, int nlayers, const double *ys, double *uvw) {
  int rc = check_call(c);
  if (rc) return rc;
  if (!eta || !psi || !uvw || !aligned16(eta) || !aligned16(psi) || !aligned16(uvw))
    return fail(c, ZK_EINVAL, "null or misaligned field pointer");
  if (nlayers < 1 || nlayers > 4096 || !ys) return fail(c, ZK_EINVAL, "nlayers must be in [1, 4096] with depths");
  for (int i = 0; i < nlayers; ++i)
    if (!std::isfinite(ys[i]) || ys[i] < 0.0 || (c->pp.depth > 0 && ys[i] > c->pp.depth))
      return fail(c, ZK_EINVAL, "layer depths must lie in [0, depth]");
  if ((rc = upload(c, c->have_plan ? c->plan_dt : NAN))) return rc;
  Phys ph;
  ph.in0 = eta;
  ph.in1 = psi;
  if (c->bc) {
    if ((rc = mirror_in(c, eta, 0)) || (rc = mirror_in(c, psi, 1))) return rc;
    ph.in0 = ext(c, 0);
    ph.in1 = ext(c, 1);
  }
  if ((rc = run_seq(c, c->plan.lift_phi, ph))) return rc;
  // chunks of layers, one column and one row launch each; with walls one
  // layer at a time through the doubled fields ext(0..2), cropped
  const size_t plane = (size_t)c->unx * c->uny;
  const int lc = c->bc ? 1 : c->plan.depth_chunk_max;
  double *ydev = reinterpret_cast<double *>(c->ws + c->off_layer);
  for (int i0 = 0; i0 < nlayers; i0 += lc) {
    const int r = std::min(lc, nlayers - i0);
    LayerDepths y{};
    for (int i = 0; i < r; ++i) y.v[i] = ys[i0 + i];
    HIP_TRY(c, launch_set_layer_depths(ydev, y, c->stream));
    ph.out0 = c->bc ? ext(c, 0) : uvw + 3 * (size_t)i0 * plane;
    if ((rc = run_seq(c, c->plan.depth_chunk[r], ph))) return rc;
    if (c->bc)
      for (int k = 0; k < 3; ++k)
        if ((rc = crop_out(c, k, uvw + (3 * (size_t)i0 + k) * plane))) return rc;
  }
  return ZK_OK;
}

int zk_autotune(zk_ctx *c, double dt, int reps) {
  int rc = check_call(c);
  if (rc) return rc;
  if (!std::isfinite(dt) || reps < 1) return fail(c, ZK_EINVAL, "dt must be finite and reps >= 1");
  if ((rc = upload(c, dt))) return rc;
  const bool prof = c->prof;
  c->prof = false;
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  for (int row = 1; row >= 0; --row)
    for (int pad = 1; pad >= 0; --pad) {
      std::vector<Launch> sub;
      for (const Launch &l : c->plan.step_body[0]) {
        const bool lr = l.kind == L_ROW_PAD || l.kind == L_ROW_BASE;
        const bool lp = l.kind == L_ROW_PAD || l.kind == L_COL_PAD;
        if (l.kind != L_PARSEVAL && lr == (bool)row && lp == (bool)pad) sub.push_back(l);
      }
      if (sub.empty() || (!row && c->pp.ny == 1)) continue;  // a 1D grid's columns have one shape
      const int n = row ? c->pp.nx : c->pp.ny;
      const int N = pad ? 3 * n / 2 : n;
      float best = 1e30f;
      int bestT = 0;
      int cand[3];
      const int ncand = radix_candidates(n, pad, cand);
      for (int ci = 0; ci < ncand; ++ci) {
        const int E = cand[ci];
        const int T = N / E;
        if (N % E || T < 2 || T > 1024 || (T & (T - 1))) continue;
        const void *fn = c->precision == 32
                             ? (row ? batch_row_kernel<float>(T, E, pad) : batch_col_kernel<float>(T, E, pad))
                             : (row ? batch_row_kernel<double>(T, E, pad) : batch_col_kernel<double>(T, E, pad));
        if (!fn) continue;
        c->tuneT[row][pad] = T;
        float tot = 0.f;
        for (int r = 0; r <= reps; ++r) {  // r = 0 warms up
          HIP_TRY(c, hipEventRecord(e0, c->stream));
          if ((rc = run_seq(c, sub, Phys{}))) return rc;
          HIP_TRY(c, hipEventRecord(e1, c->stream));
          HIP_TRY(c, hipEventSynchronize(e1));
          float ms = 0.f;
          HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
          if (r) tot += ms;
        }
        if (tot < best) {
          best = tot;
          bestT = T;
        }
      }
      c->tuneT[row][pad] = bestT;
      // padded rows: the permuted-layout transforms at the chosen shape, kept if faster
      if (row && pad && bestT && row_lanes_ok(bestT, N / bestT, true, c->precision == 32 ? 4 : 8)) {
        const int keep = c->row_fft;
        c->row_fft = ZK_ROW_FFT_LANES;
        float tot = 0.f;
        for (int r = 0; r <= reps; ++r) {
          HIP_TRY(c, hipEventRecord(e0, c->stream));
          if ((rc = run_seq(c, sub, Phys{}))) return rc;
          HIP_TRY(c, hipEventRecord(e1, c->stream));
          HIP_TRY(c, hipEventSynchronize(e1));
          float ms = 0.f;
          HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
          if (r) tot += ms;
        }
        c->row_fft = tot < best ? ZK_ROW_FFT_LANES : (keep == ZK_ROW_FFT_LANES ? ZK_ROW_FFT_STOCKHAM : keep);
      }
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->prof = prof;
  return ZK_OK;
}

int zk_team_shape(const zk_ctx *c, int row, int pad, int *T, int *E) {
  if (!c || !T || !E) return ZK_EINVAL;
  const TeamShape sh = ctx_team(c, row != 0, pad != 0);
  *T = sh.T;
  *E = sh.E;
  return ZK_OK;
}

int zk_set_team_shape(zk_ctx *c, int row, int pad, int T) {
  if (!c) return ZK_EINVAL;
  c->err.clear();
  row = row != 0;
  pad = pad != 0;
  if (T == 0) {  // back to the default shape
    c->tuneT[row][pad] = 0;
    return ZK_OK;
  }
  const int n = row ? c->pp.nx : c->pp.ny;
  const int N = pad ? 3 * n / 2 : n;
  if (!row && n == 1) return fail(c, ZK_EINVAL, "a 1D grid's column passes have no team shape");
  if (T < 2 || T > 1024 || (T & (T - 1)) || N % T) return fail(c, ZK_EINVAL, "team size must divide the transform length");
  const int E = N / T;
  const void *fn = c->precision == 32 ? (row ? batch_row_kernel<float>(T, E, pad) : batch_col_kernel<float>(T, E, pad))
                                      : (row ? batch_row_kernel<double>(T, E, pad) : batch_col_kernel<double>(T, E, pad));
  int cand[3];
  const int ncand = radix_candidates(n, pad, cand);
  if (!fn || std::find(cand, cand + ncand, E) == cand + ncand) return fail(c, ZK_EINVAL, "team shape not built");
  c->tuneT[row][pad] = T;
  return ZK_OK;
}

const char *zk_last_error(const zk_ctx *c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

// ---- allocation-free stepping ----------------------------------------------
// A file-scope device array stands in for the caller's workspace.  Each GPU
// that runs zk_step_static holds its own copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns on
// that device (the array's name in host code is not a device address).
namespace {
__device__ __align__(256) char scratch[ZK_STATIC_WS_BYTES];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

int scratch_on_device(zk_ctx *c, int dev, char **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(c, ZK_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    if (!p || ((uintptr_t)p % kAlign) != 0) return fail(c, ZK_EDEVICE, "scratch array is not 256-byte aligned");
    scratch_ptr[dev] = p;
  }
  *out = static_cast<char *>(scratch_ptr[dev]);
  return ZK_OK;
}
}  // namespace

extern "C" int zk_step_static(zk_ctx *c, double *eta, double *psi, double dt, int nsteps, void *stream) {
  if (!c) return ZK_EINVAL;
  c->err.clear();
  if (c->total > (size_t)ZK_STATIC_WS_BYTES)
    return fail(c, ZK_ENOWS, "grid needs " + std::to_string(c->total) + " workspace bytes; the static scratch holds " +
                                 std::to_string((size_t)ZK_STATIC_WS_BYTES) + " (use zk_bind and zk_step)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
  char *ws = nullptr;
  int rc = scratch_on_device(c, dev, &ws);
  if (rc) return rc;
  // Borrow the scratch for this call: the context's tables and schedules are
  // uploaded into it (another context may have left its own there), then the
  // caller's own binding, if any, is restored and marked for re-upload.
  char *ws0 = c->ws;
  const size_t bytes0 = c->ws_bytes;
  hipStream_t stream0 = c->stream;
  const int dev0 = c->device;
  const bool bound0 = c->bound, prof0 = c->prof;
  c->ws = ws;
  c->ws_bytes = ZK_STATIC_WS_BYTES;
  c->stream = static_cast<hipStream_t>(stream);
  c->device = dev;
  c->bound = true;
  c->dirty = true;
  c->have_plan = false;
  c->prof = false;  // no timing events inside this call
  rc = zk_step(c, eta, psi, dt, nsteps);
  c->ws = ws0;
  c->ws_bytes = bytes0;
  c->stream = stream0;
  c->device = dev0;
  c->bound = bound0;
  c->prof = prof0;
  c->dirty = true;
  c->have_plan = false;
  return rc;
}
