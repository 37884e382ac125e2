// zk_col_f64.hip -- col-pass kernel instances for double transforms.
#include "zk_kernels.hpp"

namespace zk {

template <>
hipError_t launch_col<double>(const ColArgs<double> &a, int T, int E, int nblocks, int nsub, hipStream_t s) {
  const dim3 grid(nblocks, nsub);
  if (T == 32 && E == 3) {
    hipLaunchKernelGGL((col_kernel<double, 32, 3>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 32 && E == 2) {
    hipLaunchKernelGGL((col_kernel<double, 32, 2>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 64 && E == 3) {
    hipLaunchKernelGGL((col_kernel<double, 64, 3>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 64 && E == 2) {
    hipLaunchKernelGGL((col_kernel<double, 64, 2>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 128 && E == 3) {
    hipLaunchKernelGGL((col_kernel<double, 128, 3>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 128 && E == 2) {
    hipLaunchKernelGGL((col_kernel<double, 128, 2>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 3) {
    hipLaunchKernelGGL((col_kernel<double, 256, 3>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 6) {
    hipLaunchKernelGGL((col_kernel<double, 256, 6>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 12) {
    hipLaunchKernelGGL((col_kernel<double, 256, 12>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 2) {
    hipLaunchKernelGGL((col_kernel<double, 256, 2>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 4) {
    hipLaunchKernelGGL((col_kernel<double, 256, 4>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 8) {
    hipLaunchKernelGGL((col_kernel<double, 256, 8>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace zk
