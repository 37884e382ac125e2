// zk_closure.hip -- pointwise and reduction kernels of the learned-closure
// stepper: FP64 sums of squares (two fixed-order stages), the network's
// input features and output scaling, the RK4 stage combinations on the grid,
// and periodic crops of training samples.  One thread per grid point; every
// index is < n (or inside the crop geometry checked by the host).
#include "zk_closure.hpp"

namespace zk {
namespace clo {
namespace {

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ double rms_of(const double *sum, long long n) {
  const double s = sqrt(sum[0] / (double)n);
  return s > 0.0 ? s : 1.0;
}

__global__ __launch_bounds__(256) void sumsq_partial(const double *__restrict__ a, const double *__restrict__ b,
                                                     long long n, double *__restrict__ part) {
  __shared__ double r0[256], r1[256];
  double s0 = 0.0, s1 = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    if (b) {
      const double d = a[i] - b[i];
      s0 += d * d;
      s1 += b[i] * b[i];
    } else {
      s0 += a[i] * a[i];
    }
  }
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      r0[threadIdx.x] += r0[threadIdx.x + o];
      r1[threadIdx.x] += r1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = r0[0];
    part[kRedBlocks + blockIdx.x] = r1[0];
  }
}

// One wavefront per sum: lane l adds the partials l, l + 64, ... in order,
// then a butterfly over the lanes (fixed order: the same bits every run).
__global__ __launch_bounds__(128) void sumsq_final(const double *__restrict__ part, double *__restrict__ out) {
  const int which = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i = lane; i < kRedBlocks; i += 64) s += part[which * kRedBlocks + i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) out[which] = s;
}

__global__ __launch_bounds__(256) void pack_kernel(const double *__restrict__ eta, const double *__restrict__ psi,
                                                   const double *__restrict__ g2, const double *__restrict__ sum,
                                                   long long n, double c_eta, double k0, uint16_t *__restrict__ xin) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double s = rms_of(sum, n);
  typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
  u16x4 v;
  v[0] = f2bf((float)(c_eta * eta[i]));
  v[1] = f2bf((float)(k0 * psi[i] / s));
  v[2] = f2bf((float)(g2[i] / s));
  v[3] = 0;
  *reinterpret_cast<u16x4 *>(xin + i * 4) = v;
}

__global__ __launch_bounds__(256) void unpack_kernel(const double *__restrict__ g2, const float *__restrict__ y,
                                                     const double *__restrict__ sum, long long n, double out_scale,
                                                     double *__restrict__ gt) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  gt[i] = g2[i] + out_scale * rms_of(sum, n) * (double)y[i];
}

__global__ __launch_bounds__(256) void features_kernel(const double *__restrict__ eta, const double *__restrict__ psi,
                                                       const double *__restrict__ g2, const double *__restrict__ g6,
                                                       const double *__restrict__ sum, long long n, double c_eta,
                                                       double k0, double out_scale, float *__restrict__ smp) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double s = rms_of(sum, n);
  smp[i] = (float)(c_eta * eta[i]);
  smp[n + i] = (float)(k0 * psi[i] / s);
  smp[2 * n + i] = (float)(g2[i] / s);
  smp[3 * n + i] = (float)((g6[i] - g2[i]) / (out_scale * s));
}

__global__ __launch_bounds__(256) void stage_kernel(const double *__restrict__ ue, const double *__restrict__ up,
                                                    const double *__restrict__ ke, const double *__restrict__ kp,
                                                    double c, double w, int first, double *__restrict__ se,
                                                    double *__restrict__ sp, double *__restrict__ ae,
                                                    double *__restrict__ ap, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double a = ke[i], b = kp[i];
  se[i] = ue[i] + c * a;
  sp[i] = up[i] + c * b;
  ae[i] = first ? w * a : ae[i] + w * a;
  ap[i] = first ? w * b : ap[i] + w * b;
}

__global__ __launch_bounds__(256) void finish_kernel(double *__restrict__ ue, double *__restrict__ up,
                                                     const double *__restrict__ ae, const double *__restrict__ ap,
                                                     const double *__restrict__ ke, const double *__restrict__ kp,
                                                     double h, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  ue[i] += h * (ae[i] + ke[i]);
  up[i] += h * (ap[i] + kp[i]);
}

__global__ __launch_bounds__(256) void crops_kernel(const float *__restrict__ src, int H, int W,
                                                    const int *__restrict__ offs, int h, int w,
                                                    float *__restrict__ dst, long long total) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int x = (int)(i % w);
  long long r = i / w;
  const int y = (int)(r % h);
  r /= h;
  const int c = (int)(r % 4);
  const long long k = r / 4;
  const int gy = (offs[2 * k] + y) % H, gx = (offs[2 * k + 1] + x) % W;  // offsets are in [0, H) x [0, W)
  dst[i] = src[(long long)c * H * W + (long long)gy * W + gx];
}

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t sumsq(const double *a, const double *b, long long n, double *part, double *out, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_partial, dim3(kRedBlocks), dim3(256), 0, s, a, b, n, part);
  hipLaunchKernelGGL(sumsq_final, dim3(1), dim3(128), 0, s, (const double *)part, out);
  return hipGetLastError();
}
hipError_t pack(const double *eta, const double *psi, const double *g2, const double *sum, long long n, double c_eta,
                double k0, uint16_t *xin, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(n)), dim3(256), 0, s, eta, psi, g2, sum, n, c_eta, k0, xin);
  return hipGetLastError();
}
hipError_t unpack(const double *g2, const float *y, const double *sum, long long n, double out_scale, double *gt,
                  hipStream_t s) {
  hipLaunchKernelGGL(unpack_kernel, dim3(blocks_for(n)), dim3(256), 0, s, g2, y, sum, n, out_scale, gt);
  return hipGetLastError();
}
hipError_t features(const double *eta, const double *psi, const double *g2, const double *g6, const double *sum,
                    long long n, double c_eta, double k0, double out_scale, float *smp, hipStream_t s) {
  hipLaunchKernelGGL(features_kernel, dim3(blocks_for(n)), dim3(256), 0, s, eta, psi, g2, g6, sum, n, c_eta, k0,
                     out_scale, smp);
  return hipGetLastError();
}
hipError_t stage(const double *ue, const double *up, const double *ke, const double *kp, double c, double w, int first,
                 double *se, double *sp, double *ae, double *ap, long long n, hipStream_t s) {
  hipLaunchKernelGGL(stage_kernel, dim3(blocks_for(n)), dim3(256), 0, s, ue, up, ke, kp, c, w, first, se, sp, ae, ap,
                     n);
  return hipGetLastError();
}
hipError_t finish(double *ue, double *up, const double *ae, const double *ap, const double *ke, const double *kp,
                  double h, long long n, hipStream_t s) {
  hipLaunchKernelGGL(finish_kernel, dim3(blocks_for(n)), dim3(256), 0, s, ue, up, ae, ap, ke, kp, h, n);
  return hipGetLastError();
}
hipError_t crops(const float *src, int H, int W, const int *offs, int ncrop, int h, int w, float *dst,
                 hipStream_t s) {
  const long long total = (long long)ncrop * 4 * h * w;
  hipLaunchKernelGGL(crops_kernel, dim3(blocks_for(total)), dim3(256), 0, s, src, H, W, offs, h, w, dst, total);
  return hipGetLastError();
}

}  // namespace clo
}  // namespace zk
