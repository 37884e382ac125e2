// zk_cnn.hpp -- closure network kernels: four circular 3 x 3 convolutions
// 3 -> 32 -> 32 -> 32 -> 1 with GELU after the first three, bf16 operands and
// FP32 accumulation, forward and backward, masked MSE loss and Adam.
//
// Device layouts (P = B*H*W pixels, pixel p = (b*H + y)*W + x):
//   samples  float  [B][4][H][W]: planes 0..2 the network input, plane 3 the
//            training target (caller-owned)
//   xin      bf16   [P][4]   input channels 0..2, channel 3 zero
//   z1..z3   float  [P][32]  pre-activations (kept for the backward pass)
//   a1..a3   bf16   [P][32]  GELU(z)
//   taps     float  [P][12]  layer 4's per-tap partial sums sum_c W4[tap][c] a3[p][c]
//            (taps 0..8; slots 9..11 unused)
//   y        float  [P]      output
//   dz4      bf16   [P]      d loss / d y
//   dz1..dz3 bf16   [P][32]  d loss / d z
//   weights  master FP32 vector in the order W1 b1 W2 b2 W3 b3 W4 b4 with
//            W (C_out, C_in, 3, 3); derived copies:
//              w1m  bf16  [co][48]        layer 1's MFMA operand, K = tap * 4 + ci
//                                          (ci = 3 and taps 9..11 zero)
//              w2f  bf16  [co][tap][ci]   forward operand of layer 2 (w3f: 3)
//              w2b  bf16  [ci][tap'][co]  backward-data operand, tap' = 8 - tap
//              w4f  float [tap][c]        (bf16-rounded values; backward)
//              w4m  bf16  [32][2][16]     layer 4's MFMA operand: row = tap (rows
//                                          9..31 zero), chunk q, K slot 8 h + j
//                                          holding channel 16 q + 8 (j / 4) + 4 h + j % 4
//   bf16 values are stored as their upper 16 bits (uint16_t).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zk {
namespace cnn {

constexpr int CH = 32;
constexpr int NW1 = CH * 3 * 9, NB1 = CH, NW2 = CH * CH * 9, NB2 = CH, NW3 = NW2, NB3 = CH, NW4 = CH * 9, NB4 = 1;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + NW1;
constexpr int OFF_W2 = OFF_B1 + NB1;
constexpr int OFF_B2 = OFF_W2 + NW2;
constexpr int OFF_W3 = OFF_B2 + NB2;
constexpr int OFF_B3 = OFF_W3 + NW3;
constexpr int OFF_W4 = OFF_B3 + NB3;
constexpr int OFF_B4 = OFF_W4 + NW4;
constexpr int NPARAM = OFF_B4 + NB4;

constexpr int kPartBlocks = 256;  // blocks of the weight-gradient kernels (one partial row each)
constexpr int kLossBlocks = 256;  // blocks of the loss kernel (one partial sum each)
constexpr int kConvTileX = 128;   // pixels per block along x in the MFMA convolution
constexpr int kConvRows = 4;      // fewest rows per block in the MFMA convolution
constexpr int kSegPx = 64;        // pixels per segment in the MFMA weight gradient

struct Geo {
  int B, H, W;
  long long pixels() const { return (long long)B * H * W; }
};

hipError_t pack_samples(const float *samples, uint16_t *xin, Geo g, hipStream_t s);
hipError_t conv1_fwd(const uint16_t *xin, const uint16_t *w1m, const float *b1, float *z1, uint16_t *a1, Geo g,
                     hipStream_t s);
// Layers 2 and 3 on MFMA.  Forward: out = bf16(GELU(conv(in) + bias)), z
// (optional) = conv(in) + bias.  Backward-data: out = bf16(conv'(din) *
// GELU'(zprev)) with the flipped, channel-transposed weights.  Needs W % 32 == 0.
hipError_t conv32_fwd(const uint16_t *in, const uint16_t *wk, const float *bias, float *z, uint16_t *out, Geo g,
                      hipStream_t s);
hipError_t conv32_bwd(const uint16_t *din, const uint16_t *wkt, const float *zprev, uint16_t *dout, Geo g,
                      hipStream_t s);
// Layer 3 forward as conv32_fwd (out may be null: activations not kept) that
// also writes layer 4's per-tap partial sums; layer 4 then sums them.
hipError_t conv32_fwd_taps(const uint16_t *in, const uint16_t *wk, const float *bias, float *z, uint16_t *out,
                           const uint16_t *w4m, float *taps, Geo g, hipStream_t s);
hipError_t conv4_fwd(const float *taps, const float *b4, float *y, Geo g, hipStream_t s);
hipError_t loss_grad(const float *y, const float *samples, int halo, double inv_n, uint16_t *dz4, double *partial,
                     Geo g, hipStream_t s);
hipError_t conv4_bwd(const uint16_t *dz4, const float *w4f, const float *z3, uint16_t *dz3, Geo g, hipStream_t s);
// Weight-gradient partial sums: part[block][W..., b...] in the flat parameter
// order of the layer; reduce_parts sums them over blocks in a fixed order.
hipError_t dw4(const uint16_t *dz4, const uint16_t *a3, float *part, Geo g, hipStream_t s);
hipError_t dw32(const uint16_t *dz, const uint16_t *a, float *part, Geo g, hipStream_t s);  // needs W % 64 == 0
hipError_t dw1(const uint16_t *dz1, const uint16_t *xin, float *part, Geo g, hipStream_t s);
hipError_t reduce_parts(const float *part, int n, float *out, hipStream_t s);
hipError_t adam(float *p, float *m, float *v, const float *g, float lr, float b1, float b2, float eps, float c1,
                float c2, hipStream_t s);
hipError_t prep_weights(const float *p, uint16_t *w1m, uint16_t *w2f, uint16_t *w2b, uint16_t *w3f, uint16_t *w3b,
                        float *w4f, uint16_t *w4m, hipStream_t s);

}  // namespace cnn
}  // namespace zk
