// zk_closure.hpp -- kernels of the learned-closure stepper (zk_closure.hip).
// Fields are FP64 [ny][nx] grids of n points.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zk {
namespace clo {

constexpr int kRedBlocks = 240;

// out[0] = sum (a - b)^2 (sum a^2 if b is null), out[1] = sum b^2 (0 if b is
// null); part holds 2 * kRedBlocks doubles.  Fixed summation order.
hipError_t sumsq(const double *a, const double *b, long long n, double *part, double *out, hipStream_t s);
// Network input [n][4] bf16: (c_eta eta, k0 psi / s, g2 / s, 0), s = rms(g2)
// from sum[0] = sum g2^2 (device).
hipError_t pack(const double *eta, const double *psi, const double *g2, const double *sum, long long n, double c_eta,
                double k0, uint16_t *xin, hipStream_t s);
// gt = g2 + out_scale * s * y.
hipError_t unpack(const double *g2, const float *y, const double *sum, long long n, double out_scale, double *gt,
                  hipStream_t s);
// Training sample [4][n] float: the three input planes of `pack` and the
// target (g6 - g2) / (out_scale * s).
hipError_t features(const double *eta, const double *psi, const double *g2, const double *g6, const double *sum,
                    long long n, double c_eta, double k0, double out_scale, float *smp, hipStream_t s);
// RK4 stage: s = u + c k; acc = (first ? 0 : acc) + w k (both fields).
hipError_t stage(const double *ue, const double *up, const double *ke, const double *kp, double c, double w, int first,
                 double *se, double *sp, double *ae, double *ap, long long n, hipStream_t s);
// u += h (acc + k).
hipError_t finish(double *ue, double *up, const double *ae, const double *ap, const double *ke, const double *kp,
                  double h, long long n, hipStream_t s);
// dst[k][c][y][x] = src[c][(offs[2k] + y) % H][(offs[2k+1] + x) % W], c < 4;
// offs (device) in [0, H) x [0, W).
hipError_t crops(const float *src, int H, int W, const int *offs, int ncrop, int h, int w, float *dst,
                 hipStream_t s);

}  // namespace clo
}  // namespace zk
