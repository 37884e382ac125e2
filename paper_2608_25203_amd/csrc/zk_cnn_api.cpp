// zk_cnn_api.cpp -- the closure network object: workspace layout, training
// step, gradient export and inference (C ABI in zk.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "zk.h"
#include "zk_cnn.hpp"
#include "zk_cnn_internal.hpp"

using namespace zk::cnn;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int fail(zk_cnn *n, int code, const std::string &m) {
  if (n) n->err = m;
  return code;
}
int hip_fail(zk_cnn *n, hipError_t e, const char *what) {
  return fail(n, ZK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIP_TRY(n, call)                                   \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail(n, e_, #call);   \
  } while (0)

void layout(zk_cnn *n) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t P = (size_t)n->max_pixels;
  n->o_p = take(NPARAM * 4);
  n->o_m = take(NPARAM * 4);
  n->o_v = take(NPARAM * 4);
  n->o_g = take(NPARAM * 4);
  n->o_w1m = take(CH * 48 * 2);
  n->o_w2f = take(NW2 * 2);
  n->o_w2b = take(NW2 * 2);
  n->o_w3f = take(NW3 * 2);
  n->o_w3b = take(NW3 * 2);
  n->o_w4f = take(NW4 * 4);
  n->o_w4m = take(32 * 32 * 2);
  n->o_part = take((size_t)kPartBlocks * (NW2 + NB2) * 4);
  n->o_loss = take(kLossBlocks * 8);
  n->o_xin = take(P * 4 * 2);
  for (int l = 0; l < 3; ++l) n->o_z[l] = take(P * CH * 4);
  for (int l = 0; l < 3; ++l) n->o_a[l] = take(P * CH * 2);
  n->o_taps = take(P * 12 * 4);
  n->o_y = take(P * 4);
  n->o_dz4 = take(P * 2);
  for (int l = 0; l < 3; ++l) n->o_dz[l] = take(P * CH * 2);
  n->total = off;
}

int check_geo(zk_cnn *n, int B, int H, int W, bool training) {
  if (!n) return ZK_EINVAL;
  n->err.clear();
  if (!n->bound) return fail(n, ZK_ENOWS, "workspace not bound (call zk_cnn_bind)");
  if (B < 1 || H < 3 || W < 32 || W % 32 != 0) return fail(n, ZK_EINVAL, "need B >= 1, H >= 3, W >= 32, W % 32 == 0");
  if (training && W % kSegPx != 0) return fail(n, ZK_EINVAL, "training needs W % 64 == 0");
  if ((long long)B * H * W > n->max_pixels) return fail(n, ZK_EINVAL, "B*H*W exceeds the network's max_pixels");
  hipError_t e = hipSetDevice(n->device);
  if (e != hipSuccess) return hip_fail(n, e, "hipSetDevice");
  return ZK_OK;
}

}  // namespace

// ---- internal entry points shared with the closure driver ------------------------------
namespace zk {
namespace cnn {

uint16_t *input_buffer(zk_cnn *n) { return reinterpret_cast<uint16_t *>(n->ws + n->o_xin); }

// Forward from the packed bf16 input buffer: y = CNN(x), optionally keeping
// the pre-activations for a backward pass.
int forward_packed(zk_cnn *n, float *y, Geo g, bool keep) {
  char *w = n->ws;
  auto f = [&](size_t o) { return reinterpret_cast<float *>(w + o); };
  auto h = [&](size_t o) { return reinterpret_cast<uint16_t *>(w + o); };
  const float *p = f(n->o_p);
  HIP_TRY(n, conv1_fwd(h(n->o_xin), h(n->o_w1m), p + OFF_B1, keep ? f(n->o_z[0]) : nullptr, h(n->o_a[0]), g, n->stream));
  HIP_TRY(n, conv32_fwd(h(n->o_a[0]), h(n->o_w2f), p + OFF_B2, keep ? f(n->o_z[1]) : nullptr, h(n->o_a[1]), g,
                        n->stream));
  HIP_TRY(n, conv32_fwd_taps(h(n->o_a[1]), h(n->o_w3f), p + OFF_B3, keep ? f(n->o_z[2]) : nullptr,
                             keep ? h(n->o_a[2]) : nullptr, h(n->o_w4m), f(n->o_taps), g, n->stream));
  HIP_TRY(n, conv4_fwd(f(n->o_taps), p + OFF_B4, y, g, n->stream));
  return ZK_OK;
}

int check_infer(zk_cnn *n, int H, int W) { return check_geo(n, 1, H, W, false); }

}  // namespace cnn
}  // namespace zk

namespace {

// Forward, loss and backward into the flat gradient vector (device).
int gradient(zk_cnn *n, const float *samples, Geo g, int halo, double *loss) {
  char *w = n->ws;
  auto f = [&](size_t o) { return reinterpret_cast<float *>(w + o); };
  auto h = [&](size_t o) { return reinterpret_cast<uint16_t *>(w + o); };
  if (halo < 0 || 2 * halo >= g.H || 2 * halo >= g.W) return fail(n, ZK_EINVAL, "halo leaves no interior");
  const double ninterior = (double)g.B * (g.H - 2 * halo) * (g.W - 2 * halo);
  HIP_TRY(n, pack_samples(samples, h(n->o_xin), g, n->stream));
  int rc = forward_packed(n, f(n->o_y), g, true);
  if (rc) return rc;
  double *lp = reinterpret_cast<double *>(w + n->o_loss);
  HIP_TRY(n, loss_grad(f(n->o_y), samples, halo, 1.0 / ninterior, h(n->o_dz4), lp, g, n->stream));
  float *part = f(n->o_part);
  float *grad = f(n->o_g);
  // layer 4
  HIP_TRY(n, dw4(h(n->o_dz4), h(n->o_a[2]), part, g, n->stream));
  HIP_TRY(n, reduce_parts(part, NW4 + NB4, grad + OFF_W4, n->stream));
  HIP_TRY(n, conv4_bwd(h(n->o_dz4), f(n->o_w4f), f(n->o_z[2]), h(n->o_dz[2]), g, n->stream));
  // layer 3
  HIP_TRY(n, dw32(h(n->o_dz[2]), h(n->o_a[1]), part, g, n->stream));
  HIP_TRY(n, reduce_parts(part, NW3 + NB3, grad + OFF_W3, n->stream));
  HIP_TRY(n, conv32_bwd(h(n->o_dz[2]), h(n->o_w3b), f(n->o_z[1]), h(n->o_dz[1]), g, n->stream));
  // layer 2
  HIP_TRY(n, dw32(h(n->o_dz[1]), h(n->o_a[0]), part, g, n->stream));
  HIP_TRY(n, reduce_parts(part, NW2 + NB2, grad + OFF_W2, n->stream));
  HIP_TRY(n, conv32_bwd(h(n->o_dz[1]), h(n->o_w2b), f(n->o_z[0]), h(n->o_dz[0]), g, n->stream));
  // layer 1
  HIP_TRY(n, dw1(h(n->o_dz[0]), h(n->o_xin), part, g, n->stream));
  HIP_TRY(n, reduce_parts(part, NW1 + NB1, grad + OFF_W1, n->stream));
  if (loss) {
    std::vector<double> hp(kLossBlocks);
    HIP_TRY(n, hipMemcpyAsync(hp.data(), lp, kLossBlocks * sizeof(double), hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(n, hipStreamSynchronize(n->stream));
    double s = 0.0;
    for (double v : hp) s += v;
    *loss = s / ninterior;
  }
  return ZK_OK;
}

int prep(zk_cnn *n) {
  char *w = n->ws;
  auto f = [&](size_t o) { return reinterpret_cast<float *>(w + o); };
  auto h = [&](size_t o) { return reinterpret_cast<uint16_t *>(w + o); };
  HIP_TRY(n, prep_weights(f(n->o_p), h(n->o_w1m), h(n->o_w2f), h(n->o_w2b), h(n->o_w3f), h(n->o_w3b), f(n->o_w4f), h(n->o_w4m),
                          n->stream));
  return ZK_OK;
}

}  // namespace

extern "C" {

zk_cnn *zk_cnn_create(long long max_pixels) {
  if (max_pixels < 32 * 3 || max_pixels > (1LL << 28)) return nullptr;
  zk_cnn *n = new (std::nothrow) zk_cnn();
  if (!n) return nullptr;
  n->max_pixels = max_pixels;
  layout(n);
  return n;
}

void zk_cnn_destroy(zk_cnn *n) { delete n; }

size_t zk_cnn_workspace_bytes(const zk_cnn *n) { return n ? n->total : 0; }

int zk_cnn_bind(zk_cnn *n, void *ws, size_t bytes, void *stream) {
  if (!n) return ZK_EINVAL;
  n->err.clear();
  if (!ws || ((uintptr_t)ws % kAlign) != 0) return fail(n, ZK_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < n->total) return fail(n, ZK_ENOWS, "workspace smaller than zk_cnn_workspace_bytes");
  int dev = 0;
  HIP_TRY(n, hipGetDevice(&dev));
  n->ws = static_cast<char *>(ws);
  n->stream = static_cast<hipStream_t>(stream);
  n->device = dev;
  n->bound = true;
  n->have_params = false;
  return ZK_OK;
}

int zk_cnn_set_params(zk_cnn *n, const float *params) {
  if (!n) return ZK_EINVAL;
  n->err.clear();
  if (!n->bound) return fail(n, ZK_ENOWS, "workspace not bound");
  if (!params) return fail(n, ZK_EINVAL, "null parameter vector");
  HIP_TRY(n, hipSetDevice(n->device));
  HIP_TRY(n, hipMemcpyAsync(n->ws + n->o_p, params, NPARAM * sizeof(float), hipMemcpyHostToDevice, n->stream));
  std::vector<float> zero(NPARAM, 0.0f);
  HIP_TRY(n, hipMemcpyAsync(n->ws + n->o_m, zero.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice, n->stream));
  HIP_TRY(n, hipMemcpyAsync(n->ws + n->o_v, zero.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice, n->stream));
  const int rc = prep(n);
  if (rc) return rc;
  HIP_TRY(n, hipStreamSynchronize(n->stream));  // host vectors go out of scope
  n->adam_t = 0;
  n->have_params = true;
  return ZK_OK;
}

int zk_cnn_get_params(zk_cnn *n, float *params) {
  if (!n) return ZK_EINVAL;
  n->err.clear();
  if (!n->bound || !n->have_params) return fail(n, ZK_EINVAL, "no parameters loaded");
  if (!params) return fail(n, ZK_EINVAL, "null output");
  HIP_TRY(n, hipSetDevice(n->device));
  HIP_TRY(n, hipMemcpyAsync(params, n->ws + n->o_p, NPARAM * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  HIP_TRY(n, hipStreamSynchronize(n->stream));
  return ZK_OK;
}

int zk_cnn_forward(zk_cnn *n, const float *samples, float *y, int B, int H, int W) {
  int rc = check_geo(n, B, H, W, false);
  if (rc) return rc;
  if (!n->have_params) return fail(n, ZK_EINVAL, "no parameters loaded");
  if (!samples || !y) return fail(n, ZK_EINVAL, "null pointer");
  const Geo g{B, H, W};
  HIP_TRY(n, pack_samples(samples, input_buffer(n), g, n->stream));
  return forward_packed(n, y, g, false);
}

int zk_cnn_gradient(zk_cnn *n, const float *samples, int B, int H, int W, int halo, double *loss, float *grad) {
  int rc = check_geo(n, B, H, W, true);
  if (rc) return rc;
  if (!n->have_params) return fail(n, ZK_EINVAL, "no parameters loaded");
  if (!samples || !grad) return fail(n, ZK_EINVAL, "null pointer");
  if ((rc = gradient(n, samples, Geo{B, H, W}, halo, loss))) return rc;
  HIP_TRY(n, hipMemcpyAsync(grad, n->ws + n->o_g, NPARAM * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  HIP_TRY(n, hipStreamSynchronize(n->stream));
  return ZK_OK;
}

int zk_cnn_train_step(zk_cnn *n, const float *samples, int B, int H, int W, int halo, double lr, double *loss) {
  int rc = check_geo(n, B, H, W, true);
  if (rc) return rc;
  if (!n->have_params) return fail(n, ZK_EINVAL, "no parameters loaded");
  if (!samples || !(lr > 0.0)) return fail(n, ZK_EINVAL, "null samples or lr <= 0");
  if ((rc = gradient(n, samples, Geo{B, H, W}, halo, loss))) return rc;
  n->adam_t += 1;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double c1 = 1.0 - std::pow(b1, (double)n->adam_t), c2 = 1.0 - std::pow(b2, (double)n->adam_t);
  char *w = n->ws;
  HIP_TRY(n, adam(reinterpret_cast<float *>(w + n->o_p), reinterpret_cast<float *>(w + n->o_m),
                  reinterpret_cast<float *>(w + n->o_v), reinterpret_cast<const float *>(w + n->o_g), (float)lr,
                  (float)b1, (float)b2, (float)eps, (float)c1, (float)c2, n->stream));
  return prep(n);
}

const char *zk_cnn_last_error(const zk_cnn *n) { return n ? n->err.c_str() : "null network"; }

}  // extern "C"
