// zk_col_f32.hip -- col-pass kernel instances for float transforms.
#include "zk_kernels.hpp"

namespace zk {

template <int E>
static bool col_launch_e(const ColArgs<float> &a, int T, dim3 grid, hipStream_t s) {
  switch (T) {
    case 8: hipLaunchKernelGGL((col_kernel<float, 8, E>), grid, dim3(32), 0, s, a); return true;
    case 16: hipLaunchKernelGGL((col_kernel<float, 16, E>), grid, dim3(64), 0, s, a); return true;
    case 32: hipLaunchKernelGGL((col_kernel<float, 32, E>), grid, dim3(128), 0, s, a); return true;
    case 64: hipLaunchKernelGGL((col_kernel<float, 64, E>), grid, dim3(256), 0, s, a); return true;
    case 128: hipLaunchKernelGGL((col_kernel<float, 128, E>), grid, dim3(256), 0, s, a); return true;
    case 256: hipLaunchKernelGGL((col_kernel<float, 256, E>), grid, dim3(256), 0, s, a); return true;
    default: return false;
  }
}

template <>
hipError_t launch_col<float>(const ColArgs<float> &a, int T, int E, int nblocks, int nsub, hipStream_t s) {
  const dim3 grid(nblocks, nsub);
  bool ok = false;
  if (E == 12) ok = col_launch_e<12>(a, T, grid, s);
  else if (E == 8) ok = col_launch_e<8>(a, T, grid, s);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace zk
