// zk_cnn_internal.hpp -- the network object behind the zk_cnn_* ABI and the
// calls the closure driver makes on it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "zk_cnn.hpp"

struct zk_cnn {
  long long max_pixels = 0;
  std::string err;
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  bool bound = false;
  bool have_params = false;
  long long adam_t = 0;
  // workspace byte offsets (layouts in zk_cnn.hpp)
  size_t o_p = 0, o_m = 0, o_v = 0, o_g = 0;
  size_t o_w1m = 0, o_w2f = 0, o_w2b = 0, o_w3f = 0, o_w3b = 0, o_w4f = 0, o_w4m = 0;
  size_t o_part = 0, o_loss = 0, o_xin = 0, o_z[3] = {0, 0, 0}, o_a[3] = {0, 0, 0}, o_taps = 0, o_y = 0, o_dz4 = 0,
         o_dz[3] = {0, 0, 0};
  size_t total = 0;
};

namespace zk {
namespace cnn {
// Packed bf16 input buffer [P][4] inside the network's workspace.
uint16_t *input_buffer(zk_cnn *n);
// y = CNN(input buffer) on the network's stream (keep: store pre-activations).
int forward_packed(zk_cnn *n, float *y, Geo g, bool keep);
// Geometry check for one H x W inference field (binds the device).
int check_infer(zk_cnn *n, int H, int W);
}  // namespace cnn
}  // namespace zk
