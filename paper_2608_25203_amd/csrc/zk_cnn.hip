// zk_cnn.hip -- kernels of the closure network (layouts in zk_cnn.hpp).
//
// Layers 2 and 3 (32 -> 32 channels, 3 x 3) are implicit GEMMs on the
// gfx950 matrix cores: v_mfma_f32_32x32x16_bf16 with the 32 output channels
// as the M dimension, 32 pixels of one row as N, and K = 9 taps x 32 input
// channels in chunks of 16.  Operand lane layout of that instruction: lane l
// holds A[l % 32][8 (l / 32) + 0..7] and B[8 (l / 32) + 0..7][l % 32]; the
// 16 accumulators of lane l hold D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
// The weight-gradient of those layers is a GEMM with K = pixels on the same
// instruction.  Layers 1 (3 -> 32) and 4 (32 -> 1) are too thin for the
// matrix cores and run on the vector ALUs.  Every kernel indexes only inside
// the buffers described in zk_cnn.hpp for the geometry it is given (checked
// by the host before launch); wrap-around is computed with non-negative
// modulo arithmetic.
#include "zk_cnn.hpp"

namespace zk {
namespace cnn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}
__device__ __forceinline__ int wrap(int i, int n) { return ((i % n) + n) % n; }
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

// ---- layer 1: 3 -> 32, one thread per pixel -------------------------------------
__global__ __launch_bounds__(256) void conv1_kernel(const uint16_t *__restrict__ xin, const float *__restrict__ w1f,
                                                    const float *__restrict__ b1, float *__restrict__ z1,
                                                    uint16_t *__restrict__ a1, int H, int W, long long P) {
  __shared__ float w[27 * CH];
  __shared__ float bb[CH];
  for (int i = threadIdx.x; i < 27 * CH; i += 256) w[i] = w1f[i];
  if (threadIdx.x < CH) bb[threadIdx.x] = b1[threadIdx.x];
  __syncthreads();
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const int x = (int)(p % W);
  const long long r = p / W;
  const int y = (int)(r % H);
  const long long b = r / H;
  float acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = bb[c];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int yy = wrap(y + t / 3 - 1, H), xx = wrap(x + t % 3 - 1, W);
    const u16x4 v = *reinterpret_cast<const u16x4 *>(xin + ((b * H + yy) * W + xx) * 4);
#pragma unroll
    for (int ci = 0; ci < 3; ++ci) {
      const float xv = bf2f(v[ci]);
#pragma unroll
      for (int c = 0; c < CH; ++c) acc[c] += w[(t * 3 + ci) * CH + c] * xv;
    }
  }
  if (z1) {
#pragma unroll
    for (int c = 0; c < CH; c += 4)
      *reinterpret_cast<float4 *>(z1 + p * CH + c) = make_float4(acc[c], acc[c + 1], acc[c + 2], acc[c + 3]);
  }
#pragma unroll
  for (int c = 0; c < CH; c += 8) {
    u16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = f2bf(gelu(acc[c + k]));
    *reinterpret_cast<u16x8 *>(a1 + p * CH + c) = o;
  }
}

// ---- layers 2, 3: 32 -> 32 on MFMA ------------------------------------------------
// Block: 4 wavefronts side by side along x (32 pixels each), kConvRows rows.
// Three input rows (y-1, y, y+1) over kConvTileX + 2 pixels sit in an LDS
// ring; the weights of the wavefront's A operand stay in registers.
constexpr int kLdsPx = kConvTileX + 2;
constexpr int kPxStride = 40;  // uint16 per pixel in LDS (32 + 8 padding: 80-byte rows)

template <bool BWD>
__global__ __launch_bounds__(256) void conv32_kernel(const uint16_t *__restrict__ in, const uint16_t *__restrict__ wk,
                                                     const float *__restrict__ bias, const float *__restrict__ zprev,
                                                     float *__restrict__ zout, uint16_t *__restrict__ out, int H,
                                                     int W) {
  __shared__ __attribute__((aligned(16))) uint16_t ring[3][kLdsPx * kPxStride];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int col = lane & 31, half = lane >> 5;
  const int x0 = blockIdx.x * kConvTileX;
  const int y0 = blockIdx.y * kConvRows;
  const int y1 = min(H, y0 + kConvRows);
  const long long b = blockIdx.z;
  const bool active = x0 + 32 * wv < W;  // W % 32 == 0

  u16x8 wa[9][2];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int q = 0; q < 2; ++q)
      wa[t][q] = *reinterpret_cast<const u16x8 *>(wk + (col * 9 + t) * CH + 16 * q + 8 * half);

  auto load_row = [&](int slot, int yy) {
    const int gy = wrap(yy, H);
    const uint16_t *src = in + ((b * H + gy) * (long long)W) * CH;
    for (int i = tid; i < kLdsPx * 4; i += 256) {
      const int p = i >> 2, q = i & 3;
      const int gx = (x0 - 1 + p + W) % W;
      *reinterpret_cast<u16x8 *>(&ring[slot][p * kPxStride + q * 8]) =
          *reinterpret_cast<const u16x8 *>(src + (long long)gx * CH + q * 8);
    }
  };

  load_row(0, y0 - 1);
  load_row(1, y0);
  for (int y = y0; y < y1; ++y) {
    const int j = y - y0;
    load_row((j + 2) % 3, y + 1);
    __syncthreads();
    if (active) {
      f32x16 acc = {};
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const uint16_t *rp = ring[(j + u) % 3];
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const u16x8 bv = *reinterpret_cast<const u16x8 *>(rp + (32 * wv + col + v) * kPxStride + 16 * q + 8 * half);
            acc = mfma(wa[u * 3 + v][q], bv, acc);
          }
      }
      const long long pix = (b * H + y) * (long long)W + x0 + 32 * wv + col;
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
        *reinterpret_cast<u16x4 *>(out + pix * CH + c0) = o;
      }
    }
    __syncthreads();
  }
}

// ---- layer 4: 32 -> 1 ------------------------------------------------------------
__global__ __launch_bounds__(256) void conv4_kernel(const uint16_t *__restrict__ a3, const float *__restrict__ w4f,
                                                    const float *__restrict__ b4, float *__restrict__ y, int H, int W,
                                                    long long P) {
  __shared__ float w[9 * CH];
  for (int i = threadIdx.x; i < 9 * CH; i += 256) w[i] = w4f[i];
  __syncthreads();
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
    const uint16_t *src = a3 + ((b * H + yy) * W + xx) * CH;
#pragma unroll
    for (int c0 = 0; c0 < CH; c0 += 8) {
      const u16x8 v = *reinterpret_cast<const u16x8 *>(src + c0);
#pragma unroll
      for (int k = 0; k < 8; ++k) acc += w[t * CH + c0 + k] * bf2f(v[k]);
    }
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
      const int gy = wrap(y + u - 1, H), gx = (x0 - 1 + p + W) % W;
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

__global__ __launch_bounds__(256) void prep_kernel(const float *__restrict__ p, float *__restrict__ w1f,
                                                   uint16_t *__restrict__ w2f, uint16_t *__restrict__ w2b,
                                                   uint16_t *__restrict__ w3f, uint16_t *__restrict__ w3b,
                                                   float *__restrict__ w4f) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= NPARAM) return;
  const uint16_t h = f2bf(p[i]);
  if (i >= OFF_W1 && i < OFF_W1 + NW1) {
    const int k = i - OFF_W1, co = k / 27, ci = (k / 9) % 3, t = k % 9;
    w1f[(t * 3 + ci) * CH + co] = bf2f(h);
  } else if ((i >= OFF_W2 && i < OFF_W2 + NW2) || (i >= OFF_W3 && i < OFF_W3 + NW3)) {
    const bool l2 = i < OFF_W2 + NW2;
    const int k = i - (l2 ? OFF_W2 : OFF_W3), o = k / (CH * 9), c = (k / 9) % CH, t = k % 9;
    (l2 ? w2f : w3f)[(o * 9 + t) * CH + c] = h;
    (l2 ? w2b : w3b)[(c * 9 + (8 - t)) * CH + o] = h;
  } else if (i >= OFF_W4 && i < OFF_W4 + NW4) {
    const int k = i - OFF_W4, c = k / 9, t = k % 9;
    w4f[t * CH + c] = bf2f(h);
  }
}

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t pack_samples(const float *samples, uint16_t *xin, Geo g, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(g.pixels())), dim3(256), 0, s, samples, xin, g.H, g.W, g.pixels());
  return hipGetLastError();
}
hipError_t conv1_fwd(const uint16_t *xin, const float *w1f, const float *b1, float *z1, uint16_t *a1, Geo g,
                     hipStream_t s) {
  hipLaunchKernelGGL(conv1_kernel, dim3(blocks_for(g.pixels())), dim3(256), 0, s, xin, w1f, b1, z1, a1, g.H, g.W,
                     g.pixels());
  return hipGetLastError();
}
hipError_t conv32_fwd(const uint16_t *in, const uint16_t *wk, const float *bias, float *z, uint16_t *out, Geo g,
                      hipStream_t s) {
  const dim3 grid((g.W + kConvTileX - 1) / kConvTileX, (g.H + kConvRows - 1) / kConvRows, g.B);
  hipLaunchKernelGGL(conv32_kernel<false>, grid, dim3(256), 0, s, in, wk, bias, (const float *)nullptr, z, out, g.H,
                     g.W);
  return hipGetLastError();
}
hipError_t conv32_bwd(const uint16_t *din, const uint16_t *wkt, const float *zprev, uint16_t *dout, Geo g,
                      hipStream_t s) {
  const dim3 grid((g.W + kConvTileX - 1) / kConvTileX, (g.H + kConvRows - 1) / kConvRows, g.B);
  hipLaunchKernelGGL(conv32_kernel<true>, grid, dim3(256), 0, s, din, wkt, (const float *)nullptr, zprev,
                     (float *)nullptr, dout, g.H, g.W);
  return hipGetLastError();
}
hipError_t conv4_fwd(const uint16_t *a3, const float *w4f, const float *b4, float *y, Geo g, hipStream_t s) {
  hipLaunchKernelGGL(conv4_kernel, dim3(blocks_for(g.pixels())), dim3(256), 0, s, a3, w4f, b4, y, g.H, g.W,
                     g.pixels());
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
hipError_t prep_weights(const float *p, float *w1f, uint16_t *w2f, uint16_t *w2b, uint16_t *w3f, uint16_t *w3b,
                        float *w4f, hipStream_t s) {
  hipLaunchKernelGGL(prep_kernel, dim3(blocks_for(NPARAM)), dim3(256), 0, s, p, w1f, w2f, w2b, w3f, w3b, w4f);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace zk
