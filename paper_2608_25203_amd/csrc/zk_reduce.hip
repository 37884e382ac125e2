// zk_reduce.hip -- deterministic two-stage FP64 Parseval sums over base spectra.
#include "zk_kernels.hpp"

namespace zk {

__device__ __forceinline__ double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Stage 1: block i sums elements i*per .. (i+1)*per-1 of the tiled layout
// (thread-strided inside the chunk) and writes two partials.
__global__ __launch_bounds__(kRedThreads) void parseval_partial(const cpx<double> *__restrict__ a,
                                                                const cpx<double> *__restrict__ b,
                                                                const cpx<double> *__restrict__ c,
                                                                const cpx<double> *__restrict__ d,
                                                                long long n, int ny, double *partial) {
  __shared__ double sh[kRedThreads];
  const long long per = (n + gridDim.x - 1) / gridDim.x;
  const long long i0 = (long long)blockIdx.x * per;
  const long long i1 = i0 + per < n ? i0 + per : n;
  double s1 = 0.0, s2 = 0.0;
  for (long long i = i0 + threadIdx.x; i < i1; i += kRedThreads) {
    const long long tile = i / ((long long)ny * CBB);
    const int kx = (int)(tile * CBB + (i % CBB));
    const double w = kx == 0 ? 1.0 : 2.0;
    s1 += w * (a[i].x * b[i].x + a[i].y * b[i].y);
    s2 += w * (c[i].x * d[i].x + c[i].y * d[i].y);
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s1;
    partial[2 * blockIdx.x + 1] = s2;
  }
}

// Stage 2: one block sums the partials in index order.
__global__ __launch_bounds__(kRedThreads) void parseval_final(const double *partial, int nparts, double *out) {
  __shared__ double sh[kRedThreads];
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kRedThreads) {
    s1 += partial[2 * i];
    s2 += partial[2 * i + 1];
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    out[0] = s1;
    out[1] = s2;
  }
}

hipError_t launch_parseval(const cpx<double> *a, const cpx<double> *b, const cpx<double> *c,
                           const cpx<double> *d, int ncols, int ny, double *partial, double *out,
                           hipStream_t s) {
  const long long n = (long long)ncols * ny;
  hipLaunchKernelGGL(parseval_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, c, d, n, ny, partial);
  hipLaunchKernelGGL(parseval_final, dim3(1), dim3(kRedThreads), 0, s, partial, kRedBlocks, out);
  return hipGetLastError();
}

}  // namespace zk
