// zk_closure_api.cpp -- learned-closure stepper (C ABI in zk.h).
//
// Classical RK4 on the grid with the DtN of a low-order context plus the
// network's residual, G = P_B(G^[low] psi + r), and the state filter after
// every step.  An audit compares that DtN with the full-order one on the
// current state; while its relative L2 error exceeds the tolerance the
// full-order context advances the state instead (its own spectral RK4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "zk.h"
#include "zk_closure.hpp"
#include "zk_cnn_internal.hpp"
#include "zk_ctx_internal.hpp"

using namespace zk;

struct zk_closure {
  zk_ctx *low = nullptr, *full = nullptr;
  zk_cnn *net = nullptr;
  double k0 = 1.0, eta_scale = 0.1, out_scale = 1.0;
  int nx = 0, ny = 0;
  std::string err;
  char *ws = nullptr;
  bool bound = false;
  size_t o_se = 0, o_sp = 0, o_ke = 0, o_kp = 0, o_ae = 0, o_ap = 0, o_g2 = 0, o_gt = 0, o_g6 = 0, o_y = 0,
         o_part = 0, o_sum = 0, o_offs = 0, total = 0;
  int max_crops = 4096;
  long long n_closure = 0, n_fallback = 0, n_audit = 0;
  double last_err = 0.0, max_err = 0.0;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int fail(zk_closure *c, int code, const std::string &m) {
  if (c) c->err = m;
  return code;
}
int hip_fail(zk_closure *c, hipError_t e, const char *what) {
  return fail(c, ZK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIP_TRY(c, call)                                 \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(c, e_, #call); \
  } while (0)
double *fld(zk_closure *c, size_t o) { return reinterpret_cast<double *>(c->ws + o); }
long long npts(const zk_closure *c) { return (long long)c->nx * c->ny; }

int prepare(zk_closure *c) {
  if (!c) return ZK_EINVAL;
  c->err.clear();
  if (!c->bound) return fail(c, ZK_ENOWS, "workspace not bound (call zk_closure_bind)");
  int rc = ctx_prepare(c->low);
  if (rc) return fail(c, rc, std::string("low-order context: ") + zk_last_error(c->low));
  if (c->full && (rc = ctx_prepare(c->full))) return fail(c, rc, std::string("full-order context: ") + zk_last_error(c->full));
  if ((rc = cnn::check_infer(c->net, c->ny, c->nx))) return fail(c, rc, std::string("network: ") + zk_cnn_last_error(c->net));
  if (!c->net->have_params) return fail(c, ZK_EINVAL, "network has no parameters");
  return ZK_OK;
}

// gt = G^[low] psi + r on the grid (r from the network).
int residual(zk_closure *c, const double *eta, const double *psi) {
  hipStream_t s = c->low->stream;
  const long long n = npts(c);
  Phys ph;
  ph.in0 = eta;
  ph.in1 = psi;
  ph.out0 = fld(c, c->o_g2);
  int rc = ctx_run(c->low, c->low->plan.dtn, ph);
  if (rc) return fail(c, rc, std::string("low-order DtN: ") + zk_last_error(c->low));
  double *sum = fld(c, c->o_sum);
  HIP_TRY(c, clo::sumsq(fld(c, c->o_g2), nullptr, n, fld(c, c->o_part), sum, s));
  HIP_TRY(c, clo::pack(eta, psi, fld(c, c->o_g2), sum, n, c->k0 / c->eta_scale, c->k0, cnn::input_buffer(c->net), s));
  float *y = reinterpret_cast<float *>(c->ws + c->o_y);
  if ((rc = cnn::forward_packed(c->net, y, cnn::Geo{1, c->ny, c->nx}, false)))
    return fail(c, rc, std::string("network: ") + zk_cnn_last_error(c->net));
  HIP_TRY(c, clo::unpack(fld(c, c->o_g2), y, sum, n, c->out_scale, fld(c, c->o_gt), s));
  return ZK_OK;
}

// (ke, kp) = closure RHS of (eta, psi).
int rhs(zk_closure *c, const double *eta, const double *psi, double *ke, double *kp) {
  int rc = residual(c, eta, psi);
  if (rc) return rc;
  Phys ph;
  ph.in0 = eta;
  ph.in1 = psi;
  ph.in2 = fld(c, c->o_gt);
  ph.out0 = ke;
  ph.out1 = kp;
  if ((rc = ctx_run(c->low, c->low->plan.rhs_g, ph))) return fail(c, rc, std::string("RHS: ") + zk_last_error(c->low));
  return ZK_OK;
}

int rk4_step(zk_closure *c, double *eta, double *psi, double dt) {
  hipStream_t s = c->low->stream;
  const long long n = npts(c);
  double *se = fld(c, c->o_se), *sp = fld(c, c->o_sp), *ke = fld(c, c->o_ke), *kp = fld(c, c->o_kp);
  double *ae = fld(c, c->o_ae), *ap = fld(c, c->o_ap);
  const double cs[3] = {0.5 * dt, 0.5 * dt, dt}, ws[3] = {1.0, 2.0, 2.0};
  int rc;
  for (int k = 0; k < 3; ++k) {
    if ((rc = rhs(c, k == 0 ? eta : se, k == 0 ? psi : sp, ke, kp))) return rc;
    HIP_TRY(c, clo::stage(eta, psi, ke, kp, cs[k], ws[k], k == 0, se, sp, ae, ap, n, s));
  }
  if ((rc = rhs(c, se, sp, ke, kp))) return rc;
  HIP_TRY(c, clo::finish(eta, psi, ae, ap, ke, kp, dt / 6.0, n, s));
  Phys ph;
  ph.in0 = eta;
  ph.in1 = psi;
  ph.out0 = eta;
  ph.out1 = psi;
  if ((rc = ctx_run(c->low, c->low->plan.filter, ph))) return fail(c, rc, std::string("filter: ") + zk_last_error(c->low));
  return ZK_OK;
}

// Relative L2 error of the closure DtN against the full-order DtN.
int audit(zk_closure *c, const double *eta, const double *psi, double *e) {
  hipStream_t s = c->low->stream;
  int rc = residual(c, eta, psi);
  if (rc) return rc;
  Phys ph;
  ph.in0 = eta;
  ph.in1 = psi;
  ph.out0 = fld(c, c->o_g6);
  if ((rc = ctx_run(c->full, c->full->plan.dtn, ph))) return fail(c, rc, std::string("full-order DtN: ") + zk_last_error(c->full));
  double *sum = fld(c, c->o_sum);
  HIP_TRY(c, clo::sumsq(fld(c, c->o_gt), fld(c, c->o_g6), npts(c), fld(c, c->o_part), sum + 2, s));
  double h[2] = {0.0, 0.0};
  HIP_TRY(c, hipMemcpyAsync(h, sum + 2, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  *e = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
  c->n_audit += 1;
  c->last_err = *e;
  c->max_err = (std::isnan(*e) || std::isnan(c->max_err)) ? *e + c->max_err : std::max(c->max_err, *e);  // NaN sticks
  return ZK_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

extern "C" {

zk_closure *zk_closure_create(zk_ctx *low, zk_ctx *full, zk_cnn *net, double k0, double eta_scale,
                              double out_scale) {
  if (!low || !net || !(k0 > 0) || !(eta_scale > 0) || !(out_scale > 0)) return nullptr;
  if (low->bc || (full && full->bc)) return nullptr;  // periodic grids only
  const PlanParams &a = low->pp;
  if (full) {
    const PlanParams &b = full->pp;
    if (a.nx != b.nx || a.ny != b.ny || a.Lx != b.Lx || a.Ly != b.Ly || a.depth != b.depth || a.g != b.g ||
        b.M <= a.M)
      return nullptr;
  }
  if ((long long)a.nx * a.ny > net->max_pixels || a.nx % 32 != 0) return nullptr;
  zk_closure *c = new (std::nothrow) zk_closure();
  if (!c) return nullptr;
  c->low = low;
  c->full = full;
  c->net = net;
  c->k0 = k0;
  c->eta_scale = eta_scale;
  c->out_scale = out_scale;
  c->nx = a.nx;
  c->ny = a.ny;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t f = (size_t)a.nx * a.ny * sizeof(double);
  c->o_se = take(f);
  c->o_sp = take(f);
  c->o_ke = take(f);
  c->o_kp = take(f);
  c->o_ae = take(f);
  c->o_ap = take(f);
  c->o_g2 = take(f);
  c->o_gt = take(f);
  c->o_g6 = take(f);
  c->o_y = take((size_t)a.nx * a.ny * sizeof(float));
  c->o_part = take(2 * clo::kRedBlocks * sizeof(double));
  c->o_sum = take(4 * sizeof(double));
  c->o_offs = take((size_t)c->max_crops * 2 * sizeof(int));
  c->total = off;
  return c;
}

void zk_closure_destroy(zk_closure *c) { delete c; }

size_t zk_closure_workspace_bytes(const zk_closure *c) { return c ? c->total : 0; }

int zk_closure_bind(zk_closure *c, void *ws, size_t bytes) {
  if (!c) return ZK_EINVAL;
  c->err.clear();
  if (!ws || ((uintptr_t)ws % kAlign) != 0) return fail(c, ZK_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < c->total) return fail(c, ZK_ENOWS, "workspace smaller than zk_closure_workspace_bytes");
  if (!c->low->bound || !c->net->bound || (c->full && !c->full->bound))
    return fail(c, ZK_ENOWS, "bind the contexts and the network first");
  if (c->net->stream != c->low->stream || (c->full && c->full->stream != c->low->stream))
    return fail(c, ZK_EINVAL, "contexts and network must share one stream");
  c->ws = static_cast<char *>(ws);
  c->bound = true;
  return ZK_OK;
}

int zk_closure_dtn(zk_closure *c, const double *eta, const double *psi, double *G) {
  int rc = prepare(c);
  if (rc) return rc;
  if (!eta || !psi || !G || !aligned16(eta) || !aligned16(psi) || !aligned16(G))
    return fail(c, ZK_EINVAL, "null or misaligned field pointer");
  return rhs(c, eta, psi, G, fld(c, c->o_kp));
}

int zk_closure_features(zk_closure *c, const double *eta, const double *psi, float *samples) {
  int rc = prepare(c);
  if (rc) return rc;
  if (!c->full) return fail(c, ZK_EINVAL, "features need the full-order context");
  if (!eta || !psi || !samples || !aligned16(eta) || !aligned16(psi)) return fail(c, ZK_EINVAL, "null or misaligned pointer");
  hipStream_t s = c->low->stream;
  Phys ph;
  ph.in0 = eta;
  ph.in1 = psi;
  ph.out0 = fld(c, c->o_g2);
  if ((rc = ctx_run(c->low, c->low->plan.dtn, ph))) return fail(c, rc, zk_last_error(c->low));
  ph.out0 = fld(c, c->o_g6);
  if ((rc = ctx_run(c->full, c->full->plan.dtn, ph))) return fail(c, rc, zk_last_error(c->full));
  double *sum = fld(c, c->o_sum);
  HIP_TRY(c, clo::sumsq(fld(c, c->o_g2), nullptr, npts(c), fld(c, c->o_part), sum, s));
  HIP_TRY(c, clo::features(eta, psi, fld(c, c->o_g2), fld(c, c->o_g6), sum, npts(c), c->k0 / c->eta_scale, c->k0,
                           c->out_scale, samples, s));
  return ZK_OK;
}

int zk_closure_crops(zk_closure *c, const float *samples, const int *offsets_host, int ncrop, int h, int w,
                     float *dst) {
  if (!c) return ZK_EINVAL;
  c->err.clear();
  if (!c->bound) return fail(c, ZK_ENOWS, "workspace not bound");
  if (!samples || !offsets_host || !dst || ncrop < 1 || ncrop > c->max_crops || h < 1 || w < 1 || h > c->ny ||
      w > c->nx)
    return fail(c, ZK_EINVAL, "bad crop arguments");
  for (int k = 0; k < 2 * ncrop; ++k)
    if (offsets_host[k] < 0 || offsets_host[k] >= (k % 2 ? c->nx : c->ny)) return fail(c, ZK_EINVAL, "crop offset out of range");
  hipStream_t s = c->low->stream;
  int *offs = reinterpret_cast<int *>(c->ws + c->o_offs);
  HIP_TRY(c, hipSetDevice(c->low->device));
  HIP_TRY(c, hipMemcpyAsync(offs, offsets_host, (size_t)ncrop * 2 * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(c, clo::crops(samples, c->ny, c->nx, offs, ncrop, h, w, dst, s));
  HIP_TRY(c, hipStreamSynchronize(s));  // the host offsets may change after return
  return ZK_OK;
}

int zk_closure_step(zk_closure *c, double *eta, double *psi, double dt, int nsteps, int audit_every, double tol) {
  int rc = prepare(c);
  if (rc) return rc;
  if (!eta || !psi || !aligned16(eta) || !aligned16(psi)) return fail(c, ZK_EINVAL, "null or misaligned field pointer");
  if (!std::isfinite(dt) || nsteps < 0 || audit_every < 0) return fail(c, ZK_EINVAL, "bad dt, nsteps or audit_every");
  if (audit_every > 0 && !c->full) return fail(c, ZK_EINVAL, "audits need the full-order context");
  int i = 0;
  while (i < nsteps) {
    const int chunk = audit_every > 0 ? std::min(audit_every, nsteps - i) : nsteps - i;
    bool use_closure = true;
    if (audit_every > 0) {
      double e = 0.0;
      if ((rc = audit(c, eta, psi, &e))) return rc;
      use_closure = e <= tol;
    }
    if (use_closure) {
      for (int k = 0; k < chunk; ++k)
        if ((rc = rk4_step(c, eta, psi, dt))) return rc;
      c->n_closure += chunk;
    } else {
      if ((rc = zk_step(c->full, eta, psi, dt, chunk))) return fail(c, rc, std::string("fallback: ") + zk_last_error(c->full));
      c->n_fallback += chunk;
    }
    i += chunk;
  }
  return ZK_OK;
}

int zk_closure_stats(const zk_closure *c, long long *closure_steps, long long *fallback_steps, long long *audits,
                     double *last_err, double *max_err) {
  if (!c) return ZK_EINVAL;
  if (closure_steps) *closure_steps = c->n_closure;
  if (fallback_steps) *fallback_steps = c->n_fallback;
  if (audits) *audits = c->n_audit;
  if (last_err) *last_err = c->last_err;
  if (max_err) *max_err = c->max_err;
  return ZK_OK;
}

const char *zk_closure_last_error(const zk_closure *c) { return c ? c->err.c_str() : "null closure"; }

}  // extern "C"
