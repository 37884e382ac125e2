// zk_col_f32.hip -- col-pass kernel instances for float transforms.
#include "zk_kernels.hpp"

namespace zk {

template <>
hipError_t launch_col<float>(const ColArgs<float> &a, int T, int E, int nblocks, int nsub, hipStream_t s) {
  const dim3 grid(nblocks, nsub);
  if (T == 32 && E == 3) {
    hipLaunchKernelGGL((col_kernel<float, 32, 3>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 32 && E == 2) {
    hipLaunchKernelGGL((col_kernel<float, 32, 2>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 64 && E == 3) {
    hipLaunchKernelGGL((col_kernel<float, 64, 3>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 64 && E == 2) {
    hipLaunchKernelGGL((col_kernel<float, 64, 2>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 128 && E == 3) {
    hipLaunchKernelGGL((col_kernel<float, 128, 3>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 128 && E == 2) {
    hipLaunchKernelGGL((col_kernel<float, 128, 2>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 3) {
    hipLaunchKernelGGL((col_kernel<float, 256, 3>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 6) {
    hipLaunchKernelGGL((col_kernel<float, 256, 6>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 12) {
    hipLaunchKernelGGL((col_kernel<float, 256, 12>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 2) {
    hipLaunchKernelGGL((col_kernel<float, 256, 2>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 4) {
    hipLaunchKernelGGL((col_kernel<float, 256, 4>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (T == 256 && E == 8) {
    hipLaunchKernelGGL((col_kernel<float, 256, 8>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace zk
