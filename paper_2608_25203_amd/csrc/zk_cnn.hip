// zk_cnn.hip -- kernels of the closure network (layouts in zk_cnn.hpp).
//
// Layers 2 and 3 (32 -> 32 channels, 3 x 3) are implicit GEMMs on the
// gfx950 matrix cores: v_mfma_f32_32x32x16_bf16 with the 32 output channels
// as the M dimension, 32 pixels of one row as N, and K = 9 taps x 32 input
// channels in chunks of 16.  Operand lane layout of that instruction: lane l
// holds A[l % 32][8 (l / 32) + 0..7] and B[8 (l / 32) + 0..7][l % 32]; the
// 16 accumulators of lane l hold D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
// The weight-gradient of those layers is a GEMM with K = pixels on the same
// instruction.  Layer 1 (3 -> 32) runs on the same instruction with K = 9
// taps x 4 channels (channel 3 and taps 9..11 zero) in three chunks.  Layer 4
// (32 -> 1) is split in two: the layer-3 kernel turns each pixel's 32
// activations into the 9 per-tap partial sums t[p][tap] = sum_c W4[tap][c]
// a3[p][c] (two more MFMAs, taps as the M dimension), and a small kernel sums
// y[p] = b4 + sum_tap t[p + off(tap)][tap].  GELU uses the erf
// approximation 7.1.26 of Abramowitz and Stegun (absolute error <= 1.5e-7,
// far below the bf16 rounding of the activations), branch-free.  Layer 4's
// backward-data and the weight gradients of layers 1 and 4 run on the vector
// ALUs.  Every kernel indexes only inside
// the buffers described in zk_cnn.hpp for the geometry it is given (checked
// by the host before launch); periodic wrap-around adds or subtracts one
// period (every offset is a single pixel).
#include <algorithm>

#include "zk_cnn.hpp"

namespace zk {
namespace cnn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// round to nearest even (the hardware conversion, v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// Standard normal CDF Phi(z) = (1 + erf(z / sqrt 2)) / 2 and e = exp(-z^2 / 2),
// with erf(a) = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) exp(-a^2),
// t = 1 / (1 + p a), a >= 0 (Abramowitz and Stegun 7.1.26), odd in a.
__device__ __forceinline__ float norm_cdf(float z, float &e) {
  const float u = z * 0.70710678118654752f;
  const float a = fabsf(u);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, a, 1.0f));
  const float poly =
      t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
  e = __builtin_amdgcn_exp2f(-1.44269504088896341f * a * a);
  return fmaf(0.5f, copysignf(fmaf(-poly, e, 1.0f), u), 0.5f);
}
__device__ __forceinline__ float gelu(float z) {
  float e;
  return z * norm_cdf(z, e);
}
__device__ __forceinline__ float gelu_d(float z) {  // Phi(z) + z phi(z)
  float e;
  const float c = norm_cdf(z, e);
  return fmaf(z * 0.39894228040143268f, e, c);
}
// i in [-n, 2n) wrapped into [0, n): every wrapped index here is a grid
// index plus or minus one
__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
__device__ __forceinline__ f32x16 mfma(u16x8 a, u16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                  0, 0);
}

__global__ __launch_bounds__(256) void pack_kernel(const float *__restrict__ smp, uint16_t *__restrict__ xin, int H,
                                                   int W, long long P) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const long long hw = (long long)H * W;
  const long long b = p / hw, r = p % hw;
  u16x4 v;
  v[0] = f2bf(smp[(b * 4 + 0) * hw + r]);
  v[1] = f2bf(smp[(b * 4 + 1) * hw + r]);
  v[2] = f2bf(smp[(b * 4 + 2) * hw + r]);
  v[3] = 0;
  *reinterpret_cast<u16x4 *>(xin + p * 4) = v;
}

// ---- layer 1: 3 -> 32 on MFMA --------------------------------------------------
// Each wavefront computes 32 pixels of one row (N) x 32 output channels (M);
// K = tap * 4 + channel over 48 (three chunks of 16), so a lane's 8 K values
// of a chunk are two taps' 4-channel pixel words (8 bytes each).  Block: 4
// wavefronts side by side along x.
__global__ __launch_bounds__(256) void conv1_kernel(const uint16_t *__restrict__ xin, const uint16_t *__restrict__ w1m,
                                                    const float *__restrict__ b1, float *__restrict__ z1,
                                                    uint16_t *__restrict__ a1, int H, int W) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int col = lane & 31, half = lane >> 5;
  const int x = blockIdx.x * 128 + 32 * wv + col;
  if (blockIdx.x * 128 + 32 * wv >= W) return;  // W % 32 == 0: whole wavefronts
  const int y = blockIdx.y;
  const long long b = blockIdx.z;
  f32x16 acc = {};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const u16x8 wa = *reinterpret_cast<const u16x8 *>(w1m + col * 48 + 16 * q + 8 * half);
    u16x8 bv = {};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int t = 4 * q + 2 * half + j;
      if (t < 9) {
        const int yy = wrap(y + t / 3 - 1, H), xx = wrap(x + t % 3 - 1, W);
        const u16x4 v = *reinterpret_cast<const u16x4 *>(xin + ((b * H + yy) * W + xx) * 4);
#pragma unroll
        for (int k = 0; k < 4; ++k) bv[4 * j + k] = v[k];
      }
    }
    acc = mfma(wa, bv, acc);
  }
  const long long pix = (b * H + y) * (long long)W + x;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int c0 = 8 * g + 4 * half;
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = acc[4 * g + k] + b1[c0 + k];
    if (z1) *reinterpret_cast<float4 *>(z1 + pix * CH + c0) = make_float4(v[0], v[1], v[2], v[3]);
    u16x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = f2bf(gelu(v[k]));
    *reinterpret_cast<u16x4 *>(a1 + pix * CH + c0) = o;
  }
}

// ---- layers 2, 3: 32 -> 32 on MFMA ------------------------------------------------
// Block: 4 wavefronts side by side along x (32 pixels each), `rows` rows
// (chosen by the host so that one round of blocks fills the chip).  Input
// rows (y-1, y, y+1) over kConvTileX + 2 pixels sit in a ring of four LDS
// slots; row y+2 is fetched into registers while row y is computed and
// written to the free slot afterwards, so one barrier per row covers both.
// The weights of the wavefront's A operand stay in registers.
constexpr int kLdsPx = kConvTileX + 2;
constexpr int kPxStride = 40;  // uint16 per pixel in LDS (32 + 8 padding: 80-byte rows)
constexpr int kRing = 4;
constexpr int kFetch = (kLdsPx * 4 + 255) / 256;  // 16-byte pieces of a ring row per thread

// Modes: forward (out = bf16(GELU(z)), z optional); forward of the last
// hidden layer, which also (or only: out may be null) writes layer 4's
// per-tap partial sums taps[p][12] (taps 0..8; the bf16 activations of the
// lane's 16 channels are the B operand of two MFMAs against W4, its rows the
// taps); backward-data (out = bf16(conv'(din) * GELU'(zprev))).
enum ConvMode { kFwd = 0, kFwdTaps = 1, kBwd = 2 };

template <int MODE>
__global__ __launch_bounds__(256) void conv32_kernel(const uint16_t *__restrict__ in, const uint16_t *__restrict__ wk,
                                                     const float *__restrict__ bias, const float *__restrict__ zprev,
                                                     float *__restrict__ zout, uint16_t *__restrict__ out,
                                                     const uint16_t *__restrict__ w4m, float *__restrict__ taps, int H,
                                                     int W, int rows) {
  constexpr bool BWD = MODE == kBwd;
  __shared__ __attribute__((aligned(16))) uint16_t ring[kRing][kLdsPx * kPxStride];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int col = lane & 31, half = lane >> 5;
  const int x0 = blockIdx.x * kConvTileX;
  const int y0 = blockIdx.y * rows;
  const int y1 = min(H, y0 + rows);
  const long long b = blockIdx.z;
  const bool active = x0 + 32 * wv < W;  // W % 32 == 0
  // ring pixels the active wavefronts read (32 per wavefront plus one on each side)
  const int npx = min(kLdsPx, W - x0 + 2);

  u16x8 wa[9][2];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int q = 0; q < 2; ++q)
      wa[t][q] = *reinterpret_cast<const u16x8 *>(wk + (col * 9 + t) * CH + 16 * q + 8 * half);

  // thread piece s: pixel p = (tid + 256 s) / 4 of the ring row, channels 8 q .. 8 q + 7
  auto fetch = [&](u16x8 (&r)[kFetch], int yy) {
    const uint16_t *src = in + ((b * H + wrap(yy, H)) * (long long)W) * CH;
#pragma unroll
    for (int s = 0; s < kFetch; ++s) {
      const int i = tid + 256 * s, p = i >> 2, q = i & 3;
      if (p < npx) r[s] = *reinterpret_cast<const u16x8 *>(src + (long long)wrap(x0 - 1 + p, W) * CH + q * 8);
    }
  };
  auto put = [&](const u16x8 (&r)[kFetch], int slot) {
#pragma unroll
    for (int s = 0; s < kFetch; ++s) {
      const int i = tid + 256 * s, p = i >> 2, q = i & 3;
      if (p < npx) *reinterpret_cast<u16x8 *>(&ring[slot][p * kPxStride + q * 8]) = r[s];
    }
  };

  {
    u16x8 r0[kFetch], r1[kFetch], r2[kFetch];
    fetch(r0, y0 - 1);
    fetch(r1, y0);
    fetch(r2, y0 + 1);
    put(r0, 0);
    put(r1, 1);
    put(r2, 2);
  }
  __syncthreads();
  u16x8 pre[kFetch];
  for (int y = y0; y < y1; ++y) {
    const int j = y - y0;
    const bool next = y + 1 < y1;  // row y + 1 of this block needs input row y + 2
    if (next) fetch(pre, y + 2);
    if (active) {
      f32x16 acc = {};
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const uint16_t *rp = ring[(j + u) % kRing];
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const u16x8 bv = *reinterpret_cast<const u16x8 *>(rp + (32 * wv + col + v) * kPxStride + 16 * q + 8 * half);
            acc = mfma(wa[u * 3 + v][q], bv, acc);
          }
      }
      const long long pix = (b * H + y) * (long long)W + x0 + 32 * wv + col;
      u16x8 act[2];  // kFwdTaps: this lane's bf16 activations as the B operand, chunk q = groups 2q, 2q + 1
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int c0 = 8 * g + 4 * half;
        float v[4] = {acc[4 * g], acc[4 * g + 1], acc[4 * g + 2], acc[4 * g + 3]};
        if constexpr (!BWD) {
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] += bias[c0 + k];
          if (zout) *reinterpret_cast<float4 *>(zout + pix * CH + c0) = make_float4(v[0], v[1], v[2], v[3]);
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] = gelu(v[k]);
        } else {
          const float4 zp = *reinterpret_cast<const float4 *>(zprev + pix * CH + c0);
          v[0] *= gelu_d(zp.x);
          v[1] *= gelu_d(zp.y);
          v[2] *= gelu_d(zp.z);
          v[3] *= gelu_d(zp.w);
        }
        u16x4 o;
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = f2bf(v[k]);
        if (MODE != kFwdTaps || out) *reinterpret_cast<u16x4 *>(out + pix * CH + c0) = o;
        if constexpr (MODE == kFwdTaps) {
#pragma unroll
          for (int k = 0; k < 4; ++k) act[g / 2][4 * (g % 2) + k] = o[k];
        }
      }
      if constexpr (MODE == kFwdTaps) {
        f32x16 tp = {};
#pragma unroll
        for (int q = 0; q < 2; ++q)
          tp = mfma(*reinterpret_cast<const u16x8 *>(w4m + (col * 2 + q) * 16 + 8 * half), act[q], tp);
        // rows 4 half + 0..3 (taps 0..7) and, for half 0, row 8 (tap 8)
        *reinterpret_cast<float4 *>(taps + pix * 12 + 4 * half) = make_float4(tp[0], tp[1], tp[2], tp[3]);
        if (half == 0) taps[pix * 12 + 8] = tp[4];
      }
    }
    // the slot of input row y - 1, last read in the previous row's step
    if (next) put(pre, (j + 3) % kRing);
    __syncthreads();
  }
}

// ---- layer 4: 32 -> 1, from the per-tap partial sums ---------------------------------
__global__ __launch_bounds__(256) void conv4_kernel(const float *__restrict__ taps, const float *__restrict__ b4,
                                                    float *__restrict__ y, int H, int W, long long P) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const int x = (int)(p % W);
  const long long r = p / W;
  const int yy0 = (int)(r % H);
  const long long b = r / H;
  float acc = b4[0];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int yy = wrap(yy0 + t / 3 - 1, H), xx = wrap(x + t % 3 - 1, W);
    acc += taps[((b * H + yy) * W + xx) * 12 + t];
  }
  y[p] = acc;
}

// ---- loss: masked mean squared error -----------------------------------------------
__global__ __launch_bounds__(256) void loss_kernel(const float *__restrict__ y, const float *__restrict__ smp, int halo,
                                                   double inv_n, uint16_t *__restrict__ dz4,
                                                   double *__restrict__ partial, int H, int W, long long P) {
  __shared__ double red[256];
  double s = 0.0;
  const long long hw = (long long)H * W;
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < P; p += (long long)gridDim.x * 256) {
    const int x = (int)(p % W);
    const long long r = p / W;
    const int yy = (int)(r % H);
    const long long b = r / H;
    const bool in = yy >= halo && yy < H - halo && x >= halo && x < W - halo;
    const double d = in ? (double)y[p] - (double)smp[(b * 4 + 3) * hw + (long long)yy * W + x] : 0.0;
    dz4[p] = f2bf((float)(2.0 * d * inv_n));
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ---- layer 4 backward-data: dz3 = (W4^T dz4) * GELU'(z3) ---------------------------
__global__ __launch_bounds__(256) void conv4_bwd_kernel(const uint16_t *__restrict__ dz4, const float *__restrict__ w4f,
                                                        const float *__restrict__ z3, uint16_t *__restrict__ dz3, int H,
                                                        int W, long long P) {
  __shared__ float w[9 * CH];
  for (int i = threadIdx.x; i < 9 * CH; i += 256) w[i] = w4f[i];
  __syncthreads();
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const int x = (int)(p % W);
  const long long r = p / W;
  const int yy0 = (int)(r % H);
  const long long b = r / H;
  float d[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {  // output pixel q - (u-1, v-1) read this pixel through tap (u, v)
    const int yy = wrap(yy0 - t / 3 + 1, H), xx = wrap(x - t % 3 + 1, W);
    d[t] = bf2f(dz4[(b * H + yy) * W + xx]);
  }
#pragma unroll
  for (int c0 = 0; c0 < CH; c0 += 4) {
    const float4 zp = *reinterpret_cast<const float4 *>(z3 + p * CH + c0);
    const float zz[4] = {zp.x, zp.y, zp.z, zp.w};
    u16x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float s = 0.f;
#pragma unroll
      for (int t = 0; t < 9; ++t) s += w[t * CH + c0 + k] * d[t];
      o[k] = f2bf(s * gelu_d(zz[k]));
    }
    *reinterpret_cast<u16x4 *>(dz3 + p * CH + c0) = o;
  }
}

// ---- weight gradients of layers 4 and 1 (vector ALUs) --------------------------------
// Thread t owns channel t % 32 and taps t / 32 (and tap 8 for t < 32); each
// block sums a contiguous chunk of pixels.
__global__ __launch_bounds__(256) void dw4_kernel(const uint16_t *__restrict__ dz4, const uint16_t *__restrict__ a3,
                                                  float *__restrict__ part, int H, int W, long long P) {
  const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
  const long long chunk = (P + gridDim.x - 1) / gridDim.x;
  const long long p0 = (long long)blockIdx.x * chunk, p1 = min(P, p0 + chunk);
  float acc0 = 0.f, acc8 = 0.f, accb = 0.f;
  for (long long p = p0; p < p1; ++p) {
    const float d = bf2f(dz4[p]);
    const int x = (int)(p % W);
    const long long r = p / W;
    const int y = (int)(r % H);
    const long long b = r / H;
    {
      const int yy = wrap(y + g / 3 - 1, H), xx = wrap(x + g % 3 - 1, W);
      acc0 += d * bf2f(a3[((b * H + yy) * W + xx) * CH + c]);
    }
    if (g == 0) {
      const int yy = wrap(y + 1, H), xx = wrap(x + 1, W);  // tap 8 = (2, 2)
      acc8 += d * bf2f(a3[((b * H + yy) * W + xx) * CH + c]);
      accb += d;
    }
  }
  float *o = part + (long long)blockIdx.x * (NW4 + NB4);
  o[c * 9 + g] = acc0;
  if (g == 0) o[c * 9 + 8] = acc8;
  if (threadIdx.x == 0) o[NW4] = accb;
}

__global__ __launch_bounds__(256) void dw1_kernel(const uint16_t *__restrict__ dz1, const uint16_t *__restrict__ xin,
                                                  float *__restrict__ part, int H, int W, long long P) {
  const int co = threadIdx.x & 31, g = threadIdx.x >> 5;
  const long long chunk = (P + gridDim.x - 1) / gridDim.x;
  const long long p0 = (long long)blockIdx.x * chunk, p1 = min(P, p0 + chunk);
  float a0[3] = {0.f, 0.f, 0.f}, a8[3] = {0.f, 0.f, 0.f}, accb = 0.f;
  for (long long p = p0; p < p1; ++p) {
    const float d = bf2f(dz1[p * CH + co]);
    const int x = (int)(p % W);
    const long long r = p / W;
    const int y = (int)(r % H);
    const long long b = r / H;
    {
      const int yy = wrap(y + g / 3 - 1, H), xx = wrap(x + g % 3 - 1, W);
      const u16x4 v = *reinterpret_cast<const u16x4 *>(xin + ((b * H + yy) * W + xx) * 4);
#pragma unroll
      for (int ci = 0; ci < 3; ++ci) a0[ci] += d * bf2f(v[ci]);
    }
    if (g == 0) {
      const int yy = wrap(y + 1, H), xx = wrap(x + 1, W);
      const u16x4 v = *reinterpret_cast<const u16x4 *>(xin + ((b * H + yy) * W + xx) * 4);
#pragma unroll
      for (int ci = 0; ci < 3; ++ci) a8[ci] += d * bf2f(v[ci]);
      accb += d;
    }
  }
  float *o = part + (long long)blockIdx.x * (NW1 + NB1);
#pragma unroll
  for (int ci = 0; ci < 3; ++ci) o[(co * 3 + ci) * 9 + g] = a0[ci];
  if (g == 0) {
#pragma unroll
    for (int ci = 0; ci < 3; ++ci) o[(co * 3 + ci) * 9 + 8] = a8[ci];
    o[NW1 + co] = accb;
  }
}

// ---- weight gradient of layers 2, 3 on MFMA -----------------------------------------
// dW[o][c][tap] = sum_p dz[p][o] a[p + off(tap)][c]: M = o, N = c, K = the
// 64 pixels of one row segment.  The segment's dz and the three shifted
// copies of the three activation rows are staged transposed in LDS
// (channel-major, pixels contiguous), so each operand is one 16-byte read.
constexpr int kTS = kSegPx + 8;  // uint16 stride of a transposed LDS row

__global__ __launch_bounds__(256) void dw32_kernel(const uint16_t *__restrict__ dz, const uint16_t *__restrict__ act,
                                                   float *__restrict__ part, int B, int H, int W) {
  __shared__ __attribute__((aligned(16))) uint16_t dzT[CH * kTS];
  __shared__ __attribute__((aligned(16))) uint16_t aT[9][CH * kTS];  // [u * 3 + shift][c][px]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int col = lane & 31, half = lane >> 5;
  f32x16 acc[3] = {{}, {}, {}};
  float accb = 0.f;
  const int segs_row = W / kSegPx;
  const long long nseg = (long long)B * H * segs_row;
  for (long long s = blockIdx.x; s < nseg; s += gridDim.x) {
    const int xs = (int)(s % segs_row);
    const long long r = s / segs_row;
    const int y = (int)(r % H);
    const long long b = r / H;
    const int x0 = xs * kSegPx;
    {
      const int p = tid >> 2, q = tid & 3;  // 64 pixels x 4 chunks of 8 channels
      const u16x8 v = *reinterpret_cast<const u16x8 *>(dz + ((b * H + y) * (long long)W + x0 + p) * CH + 8 * q);
#pragma unroll
      for (int k = 0; k < 8; ++k) dzT[(8 * q + k) * kTS + p] = v[k];
    }
    for (int i = tid; i < 3 * (kSegPx + 2) * 4; i += 256) {
      const int u = i / ((kSegPx + 2) * 4), rem = i % ((kSegPx + 2) * 4);
      const int p = rem >> 2, q = rem & 3;
      const int gy = wrap(y + u - 1, H), gx = wrap(x0 - 1 + p, W);
      const u16x8 v = *reinterpret_cast<const u16x8 *>(act + ((b * H + gy) * (long long)W + gx) * CH + 8 * q);
#pragma unroll
      for (int sh = 0; sh < 3; ++sh) {
        const int px = p - sh;
        if (px >= 0 && px < kSegPx) {
#pragma unroll
          for (int k = 0; k < 8; ++k) aT[u * 3 + sh][(8 * q + k) * kTS + px] = v[k];
        }
      }
    }
    __syncthreads();
    if (tid < CH) {
      for (int px = 0; px < kSegPx; ++px) accb += bf2f(dzT[tid * kTS + px]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int t = wv + 4 * k;
      if (t < 9) {
#pragma unroll
        for (int kc = 0; kc < kSegPx / 16; ++kc) {
          const u16x8 av = *reinterpret_cast<const u16x8 *>(dzT + col * kTS + 16 * kc + 8 * half);
          const u16x8 bv = *reinterpret_cast<const u16x8 *>(aT[t] + col * kTS + 16 * kc + 8 * half);
          acc[k] = mfma(av, bv, acc[k]);
        }
      }
    }
    __syncthreads();
  }
  float *o = part + (long long)blockIdx.x * (NW2 + NB2);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int t = wv + 4 * k;
    if (t < 9) {
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        const int oc = 8 * (rr / 4) + 4 * half + (rr % 4);
        o[(oc * CH + col) * 9 + t] = acc[k][rr];
      }
    }
  }
  if (tid < CH) o[NW2 + tid] = accb;
}

__global__ __launch_bounds__(256) void reduce_kernel(const float *__restrict__ part, int n, int nb,
                                                     float *__restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int b = 0; b < nb; ++b) s += part[(long long)b * n + i];
  out[i] = s;
}

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                                                   const float *__restrict__ g, float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= NPARAM) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(256) void prep_kernel(const float *__restrict__ p, uint16_t *__restrict__ w1m,
                                                   uint16_t *__restrict__ w2f, uint16_t *__restrict__ w2b,
                                                   uint16_t *__restrict__ w3f, uint16_t *__restrict__ w3b,
                                                   float *__restrict__ w4f, uint16_t *__restrict__ w4m) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  // the zero slots of the MFMA operands (channel 3 and taps 9..11 of w1m; rows 9..31 of w4m)
  if (i < CH * 48 && (i % 4 == 3 || i % 48 >= 36)) w1m[i] = 0;
  if (i >= 9 * 32 && i < 32 * 32) w4m[i] = 0;
  if (i >= NPARAM) return;
  const uint16_t h = f2bf(p[i]);
  if (i >= OFF_W1 && i < OFF_W1 + NW1) {
    const int k = i - OFF_W1, co = k / 27, ci = (k / 9) % 3, t = k % 9;
    w1m[co * 48 + t * 4 + ci] = h;
  } else if ((i >= OFF_W2 && i < OFF_W2 + NW2) || (i >= OFF_W3 && i < OFF_W3 + NW3)) {
    const bool l2 = i < OFF_W2 + NW2;
    const int k = i - (l2 ? OFF_W2 : OFF_W3), o = k / (CH * 9), c = (k / 9) % CH, t = k % 9;
    (l2 ? w2f : w3f)[(o * 9 + t) * CH + c] = h;
    (l2 ? w2b : w3b)[(c * 9 + (8 - t)) * CH + o] = h;
  } else if (i >= OFF_W4 && i < OFF_W4 + NW4) {
    const int k = i - OFF_W4, c = k / 9, t = k % 9;
    w4f[t * CH + c] = bf2f(h);
    // MFMA operand: row t, chunk c / 16, K slot 8 h + j with c % 16 = 8 (j / 4) + 4 h + j % 4
    const int q = c / 16, hh = (c % 8) / 4, j = 4 * ((c % 16) / 8) + c % 4;
    w4m[(t * 2 + q) * 16 + 8 * hh + j] = h;
  }
}

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t pack_samples(const float *samples, uint16_t *xin, Geo g, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(g.pixels())), dim3(256), 0, s, samples, xin, g.H, g.W, g.pixels());
  return hipGetLastError();
}
hipError_t conv1_fwd(const uint16_t *xin, const uint16_t *w1m, const float *b1, float *z1, uint16_t *a1, Geo g,
                     hipStream_t s) {
  const dim3 grid((g.W + 127) / 128, g.H, g.B);
  hipLaunchKernelGGL(conv1_kernel, grid, dim3(256), 0, s, xin, w1m, b1, z1, a1, g.H, g.W);
  return hipGetLastError();
}
// Rows per block of a layer-2/3 launch: enough that one round of resident
// blocks covers the grid (each block pays a three-row prologue), at least
// kConvRows.  `resident` = blocks of this kernel the whole chip holds at once.
template <int MODE>
int conv_rows(Geo g) {
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, conv32_kernel<MODE>, 256, 0) != hipSuccess)
      cus = per_cu = 0;
    resident = cus > 0 && per_cu > 0 ? cus * per_cu : 1024;
  }
  const long long strips = (long long)g.B * ((g.W + kConvTileX - 1) / kConvTileX);  // blocks per row band
  const long long need = (strips * g.H + resident - 1) / resident;
  return (int)std::min<long long>(g.H, std::max<long long>(kConvRows, need));
}
template <int MODE>
hipError_t conv32_launch(const uint16_t *in, const uint16_t *wk, const float *bias, const float *zprev, float *z,
                         uint16_t *out, const uint16_t *w4m, float *taps, Geo g, hipStream_t s) {
  const int rows = conv_rows<MODE>(g);
  const dim3 grid((g.W + kConvTileX - 1) / kConvTileX, (g.H + rows - 1) / rows, g.B);
  hipLaunchKernelGGL(conv32_kernel<MODE>, grid, dim3(256), 0, s, in, wk, bias, zprev, z, out, w4m, taps, g.H, g.W,
                     rows);
  return hipGetLastError();
}
hipError_t conv32_fwd(const uint16_t *in, const uint16_t *wk, const float *bias, float *z, uint16_t *out, Geo g,
                      hipStream_t s) {
  return conv32_launch<kFwd>(in, wk, bias, nullptr, z, out, nullptr, nullptr, g, s);
}
hipError_t conv32_fwd_taps(const uint16_t *in, const uint16_t *wk, const float *bias, float *z, uint16_t *out,
                           const uint16_t *w4m, float *taps, Geo g, hipStream_t s) {
  return conv32_launch<kFwdTaps>(in, wk, bias, nullptr, z, out, w4m, taps, g, s);
}
hipError_t conv32_bwd(const uint16_t *din, const uint16_t *wkt, const float *zprev, uint16_t *dout, Geo g,
                      hipStream_t s) {
  return conv32_launch<kBwd>(din, wkt, nullptr, zprev, nullptr, dout, nullptr, nullptr, g, s);
}
hipError_t conv4_fwd(const float *taps, const float *b4, float *y, Geo g, hipStream_t s) {
  hipLaunchKernelGGL(conv4_kernel, dim3(blocks_for(g.pixels())), dim3(256), 0, s, taps, b4, y, g.H, g.W, g.pixels());
  return hipGetLastError();
}
hipError_t loss_grad(const float *y, const float *samples, int halo, double inv_n, uint16_t *dz4, double *partial,
                     Geo g, hipStream_t s) {
  hipLaunchKernelGGL(loss_kernel, dim3(kLossBlocks), dim3(256), 0, s, y, samples, halo, inv_n, dz4, partial, g.H, g.W,
                     g.pixels());
  return hipGetLastError();
}
hipError_t conv4_bwd(const uint16_t *dz4, const float *w4f, const float *z3, uint16_t *dz3, Geo g, hipStream_t s) {
  hipLaunchKernelGGL(conv4_bwd_kernel, dim3(blocks_for(g.pixels())), dim3(256), 0, s, dz4, w4f, z3, dz3, g.H, g.W,
                     g.pixels());
  return hipGetLastError();
}
hipError_t dw4(const uint16_t *dz4, const uint16_t *a3, float *part, Geo g, hipStream_t s) {
  hipLaunchKernelGGL(dw4_kernel, dim3(kPartBlocks), dim3(256), 0, s, dz4, a3, part, g.H, g.W, g.pixels());
  return hipGetLastError();
}
hipError_t dw32(const uint16_t *dz, const uint16_t *a, float *part, Geo g, hipStream_t s) {
  hipLaunchKernelGGL(dw32_kernel, dim3(kPartBlocks), dim3(256), 0, s, dz, a, part, g.B, g.H, g.W);
  return hipGetLastError();
}
hipError_t dw1(const uint16_t *dz1, const uint16_t *xin, float *part, Geo g, hipStream_t s) {
  hipLaunchKernelGGL(dw1_kernel, dim3(kPartBlocks), dim3(256), 0, s, dz1, xin, part, g.H, g.W, g.pixels());
  return hipGetLastError();
}
hipError_t reduce_parts(const float *part, int n, float *out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(n)), dim3(256), 0, s, part, n, kPartBlocks, out);
  return hipGetLastError();
}
hipError_t adam(float *p, float *m, float *v, const float *g, float lr, float b1, float b2, float eps, float c1,
                float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(NPARAM)), dim3(256), 0, s, p, m, v, g, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t prep_weights(const float *p, uint16_t *w1m, uint16_t *w2f, uint16_t *w2b, uint16_t *w3f, uint16_t *w3b,
                        float *w4f, uint16_t *w4m, hipStream_t s) {
  hipLaunchKernelGGL(prep_kernel, dim3(blocks_for(NPARAM)), dim3(256), 0, s, p, w1m, w2f, w2b, w3f, w3b, w4f, w4m);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace zk
