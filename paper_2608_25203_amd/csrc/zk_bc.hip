// zk_bc.hip -- even extension and crop of caller fields for reflecting walls, and
// the per-layer kernels of the bulk velocity lift
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

// (C, S) of one depth layer per band element, in the stable exponential
// form of eq:CiSi_stable; C = 1, S = 0 at k = 0.
__global__ __launch_bounds__(256) void fill_layer_kernel(double *__restrict__ tab, int nx, int ny, double kxs,
                                                         double kys, double depth, double y) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= (nx / 2) * ny) return;
  const int col = i / ny, b = i % ny;
  const int my = b < ny / 2 ? b : b - ny;
  const double kx = kxs * col, ky = kys * my, k = sqrt(kx * kx + ky * ky);
  double C = 1.0, S = 0.0;
  if (k > 0.0) {
    const double e1 = exp(-k * y);
    if (depth > 0.0) {
      const double e2 = exp(-2.0 * k * (depth - y)), den = 1.0 + exp(-2.0 * k * depth);
      C = e1 * (1.0 + e2) / den;
      S = k * e1 * (1.0 - e2) / den;
    } else {
      C = e1;
      S = k * e1;
    }
  }
  const long long e = ((long long)(col / CBB) * ny + b) * CBB + col % CBB;
  tab[2 * e] = C;
  tab[2 * e + 1] = S;
}

}  // namespace

hipError_t launch_fill_layer(double *tab, int nx, int ny, double kx_scale, double ky_scale, double depth, double y,
                             hipStream_t s) {
  const int total = (nx / 2) * ny;
  hipLaunchKernelGGL(fill_layer_kernel, dim3((total + 255) / 256), dim3(256), 0, s, tab, nx, ny, kx_scale, ky_scale,
                     depth, y);
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
