// zk_row_f32.hip -- row-pass kernel instances for float transforms.
#include "zk_kernels.hpp"

namespace zk {

template <int E>
static bool row_launch_e(const RowArgs<float> &a, int T, dim3 grid, hipStream_t s) {
  switch (T) {
    case 8: hipLaunchKernelGGL((row_kernel<float, 8, E>), grid, dim3(256), 0, s, a); return true;
    case 16: hipLaunchKernelGGL((row_kernel<float, 16, E>), grid, dim3(256), 0, s, a); return true;
    case 32: hipLaunchKernelGGL((row_kernel<float, 32, E>), grid, dim3(256), 0, s, a); return true;
    case 64: hipLaunchKernelGGL((row_kernel<float, 64, E>), grid, dim3(256), 0, s, a); return true;
    case 128: hipLaunchKernelGGL((row_kernel<float, 128, E>), grid, dim3(256), 0, s, a); return true;
    case 256: hipLaunchKernelGGL((row_kernel<float, 256, E>), grid, dim3(256), 0, s, a); return true;
    default: return false;
  }
}

template <>
hipError_t launch_row<float>(const RowArgs<float> &a, int T, int E, int nblocks, int nsub, hipStream_t s) {
  const dim3 grid(nblocks, nsub);
  bool ok = false;
  if (E == 12) ok = row_launch_e<12>(a, T, grid, s);
  else if (E == 8) ok = row_launch_e<8>(a, T, grid, s);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace zk
