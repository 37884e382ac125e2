// zk_bc.hip -- even extension and crop of caller fields for reflecting walls, and
// the depths of a chunk of layers of the bulk velocity lift
// (Sec. "Boundary conditions via even extension", eq:even_ext).  The tank's
// nx x ny cell-centred field is mirrored across each wall onto the doubled
// 2nx x 2ny periodic grid, half-sample symmetric: f~(2n - 1 - i) = f(i).
// One thread per output point; every index stays inside [ny][nx] or
// [2ny][2nx].
#include "zk_kernels.hpp"

namespace zk {
namespace {

__global__ __launch_bounds__(256) void mirror_kernel(const double *__restrict__ src, int nx, int ny,
                                                     double *__restrict__ dst) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long total = 4LL * nx * ny;
  if (i >= total) return;
  const int x = (int)(i % (2 * nx)), y = (int)(i / (2 * nx));
  const int sx = x < nx ? x : 2 * nx - 1 - x;
  const int sy = y < ny ? y : 2 * ny - 1 - y;
  dst[i] = src[(long long)sy * nx + sx];
}

__global__ __launch_bounds__(256) void crop_kernel(const double *__restrict__ src, int nx, int ny,
                                                   double *__restrict__ dst) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long long)nx * ny) return;
  const int x = (int)(i % nx), y = (int)(i / nx);
  dst[i] = src[(long long)y * (2 * nx) + x];
}

__global__ void set_layer_depths_kernel(double *__restrict__ dst, LayerDepths y) {
  const int i = threadIdx.x;
  if (i < kMaxChunkLayers) dst[i] = y.v[i];
}

}  // namespace

hipError_t launch_set_layer_depths(double *dst, LayerDepths y, hipStream_t s) {
  hipLaunchKernelGGL(set_layer_depths_kernel, dim3(1), dim3(64), 0, s, dst, y);
  return hipGetLastError();
}

hipError_t launch_mirror(const double *src, int nx, int ny, double *dst, hipStream_t s) {
  const long long total = 4LL * nx * ny;
  hipLaunchKernelGGL(mirror_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, nx, ny, dst);
  return hipGetLastError();
}

hipError_t launch_crop(const double *src, int nx, int ny, double *dst, hipStream_t s) {
  const long long total = (long long)nx * ny;
  hipLaunchKernelGGL(crop_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, nx, ny, dst);
  return hipGetLastError();
}

}  // namespace zk
