// zk_batch_col_f64.hip -- batched col-pass kernel instances (double transforms);
// written by gen_batch_units.py.
#include "zk_kernels.hpp"

namespace zk {

template <>
const void *batch_col_kernel<double>(int T, int E, bool pad) {
  if (T == 2 && E == 2 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 2, 2>);
  if (T == 2 && E == 3 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 2, 3>);
  if (T == 2 && E == 4 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 2, 4>);
  if (T == 2 && E == 6 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 2, 6>);
  if (T == 4 && E == 2 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 4, 2>);
  if (T == 4 && E == 3 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 4, 3>);
  if (T == 4 && E == 4 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 4, 4>);
  if (T == 4 && E == 6 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 4, 6>);
  if (T == 8 && E == 2 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 8, 2>);
  if (T == 8 && E == 3 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 8, 3>);
  if (T == 8 && E == 4 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 8, 4>);
  if (T == 8 && E == 6 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 8, 6>);
  if (T == 16 && E == 2 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 16, 2>);
  if (T == 16 && E == 3 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 16, 3>);
  if (T == 16 && E == 4 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 16, 4>);
  if (T == 16 && E == 6 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 16, 6>);
  if (T == 32 && E == 2 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 32, 2>);
  if (T == 32 && E == 3 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 32, 3>);
  if (T == 32 && E == 4 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 32, 4>);
  if (T == 32 && E == 6 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 32, 6>);
  if (T == 32 && E == 8 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 32, 8>);
  if (T == 32 && E == 12 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 32, 12>);
  if (T == 64 && E == 2 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 64, 2>);
  if (T == 64 && E == 3 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 64, 3>);
  if (T == 64 && E == 4 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 64, 4>);
  if (T == 64 && E == 6 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 64, 6>);
  if (T == 64 && E == 8 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 64, 8>);
  if (T == 64 && E == 12 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 64, 12>);
  if (T == 128 && E == 2 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 128, 2>);
  if (T == 128 && E == 3 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 128, 3>);
  if (T == 128 && E == 4 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 128, 4>);
  if (T == 128 && E == 6 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 128, 6>);
  if (T == 128 && E == 8 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 128, 8>);
  if (T == 128 && E == 12 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 128, 12>);
  if (T == 256 && E == 2 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 256, 2>);
  if (T == 256 && E == 3 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 256, 3>);
  if (T == 256 && E == 4 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 256, 4>);
  if (T == 256 && E == 6 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 256, 6>);
  if (T == 256 && E == 8 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 256, 8>);
  if (T == 256 && E == 12 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 256, 12>);
  if (T == 512 && E == 2 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 512, 2>);
  if (T == 512 && E == 3 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 512, 3>);
  if (T == 512 && E == 4 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 512, 4>);
  if (T == 512 && E == 6 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 512, 6>);
  if (T == 1024 && E == 2 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 1024, 2>);
  if (T == 1024 && E == 3 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 1024, 3>);
  if (T == 2 && E == 9 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 2, 9>);
  if (T == 4 && E == 9 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 4, 9>);
  if (T == 8 && E == 9 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 8, 9>);
  if (T == 16 && E == 9 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 16, 9>);
  if (T == 32 && E == 9 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 32, 9>);
  if (T == 64 && E == 9 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 64, 9>);
  if (T == 128 && E == 9 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 128, 9>);
  if (T == 256 && E == 9 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 256, 9>);
  if (T == 2 && E == 6 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 2, 6, false, false>);
  if (T == 4 && E == 6 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 4, 6, false, false>);
  if (T == 8 && E == 6 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 8, 6, false, false>);
  if (T == 16 && E == 6 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 16, 6, false, false>);
  if (T == 32 && E == 6 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 32, 6, false, false>);
  if (T == 64 && E == 6 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 64, 6, false, false>);
  if (T == 128 && E == 6 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 128, 6, false, false>);
  if (T == 256 && E == 6 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 256, 6, false, false>);
  if (T == 2 && E == 15 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 2, 15>);
  if (T == 4 && E == 15 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 4, 15>);
  if (T == 8 && E == 15 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 8, 15>);
  if (T == 16 && E == 15 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 16, 15>);
  if (T == 32 && E == 15 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 32, 15>);
  if (T == 64 && E == 15 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 64, 15>);
  if (T == 128 && E == 15 && pad == true) return reinterpret_cast<const void *>(&col_kernel_batch<double, 128, 15>);
  if (T == 2 && E == 10 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 2, 10>);
  if (T == 4 && E == 10 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 4, 10>);
  if (T == 8 && E == 10 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 8, 10>);
  if (T == 16 && E == 10 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 16, 10>);
  if (T == 32 && E == 10 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 32, 10>);
  if (T == 64 && E == 10 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 64, 10>);
  if (T == 128 && E == 10 && pad == false) return reinterpret_cast<const void *>(&col_kernel_batch<double, 128, 10>);
  return nullptr;
}

template <>
hipError_t launch_batch_col<double>(int T, int E, bool pad, dim3 grid, hipStream_t s, const ColArgs<double> *args,
                                   const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph) {
  if (T == 2 && E == 2 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 2 && E == 3 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 2 && E == 4 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 2 && E == 6 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 2 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 3 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 4 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 6 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 2 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 3 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 4 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 6 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 2 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 3 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 4 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 6 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 2 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 3 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 4 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 6 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 8 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 8>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 12 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 12>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 2 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 3 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 4 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 6 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 8 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 8>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 12 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 12>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 2 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 3 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 4 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 6 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 8 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 8>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 12 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 12>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 2 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 3 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 4 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 6 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 8 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 8>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 12 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 12>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 2 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 512, 2>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 3 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 512, 3>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 4 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 512, 4>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 6 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 512, 6>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 1024 && E == 2 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 1024, 2>), grid, dim3(1024), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 1024 && E == 3 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 1024, 3>), grid, dim3(1024), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 2 && E == 9 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 9>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 9 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 9>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 9 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 9>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 9 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 9>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 9 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 9>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 9 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 9>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 9 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 9>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 9 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 9>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 2 && E == 6 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 6, false, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 6 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 6, false, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 6 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 6, false, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 6 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 6, false, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 6 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 6, false, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 6 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 6, false, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 6 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 6, false, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 6 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 6, false, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 2 && E == 15 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 15>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 15 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 15>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 15 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 15>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 15 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 15>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 15 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 15>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 15 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 15>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 15 && pad == true) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 15>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 2 && E == 10 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 10>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 10 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 10>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 10 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 10>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 10 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 10>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 10 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 10>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 10 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 10>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 10 && pad == false) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 10>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_batch_col_lift<double>(int T, int E, dim3 grid, hipStream_t s, const ColArgs<double> *args,
                                        const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph) {
  if (T == 2 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 2 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 8, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 8, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 8, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 8, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<double, 512, 2, true>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<double, 512, 4, true>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 1024 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<double, 1024, 2, true>), grid, dim3(1024), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 2 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 6, true, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 6, true, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 6, true, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 6, true, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 6, true, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 6, true, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 6, true, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<double, 256, 6, true, false>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 2 && E == 10) {
    hipLaunchKernelGGL((col_kernel_batch<double, 2, 10, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 4 && E == 10) {
    hipLaunchKernelGGL((col_kernel_batch<double, 4, 10, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 8 && E == 10) {
    hipLaunchKernelGGL((col_kernel_batch<double, 8, 10, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 16 && E == 10) {
    hipLaunchKernelGGL((col_kernel_batch<double, 16, 10, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 10) {
    hipLaunchKernelGGL((col_kernel_batch<double, 32, 10, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 10) {
    hipLaunchKernelGGL((col_kernel_batch<double, 64, 10, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 10) {
    hipLaunchKernelGGL((col_kernel_batch<double, 128, 10, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_batch_col_folds<double>(int T, int E, dim3 grid, hipStream_t s, const ColArgs<double> *args,
                                         const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph) {
  if (T == 64 && E == 2) {
    hipLaunchKernelGGL((col_kernel_folds<double, 64, 2>), grid, dim3(kMaxFolds * 64), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 3) {
    hipLaunchKernelGGL((col_kernel_folds<double, 64, 3>), grid, dim3(kMaxFolds * 64), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 2) {
    hipLaunchKernelGGL((col_kernel_folds<double, 128, 2>), grid, dim3(kMaxFolds * 128), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 3) {
    hipLaunchKernelGGL((col_kernel_folds<double, 128, 3>), grid, dim3(kMaxFolds * 128), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 2) {
    hipLaunchKernelGGL((col_kernel_folds<double, 256, 2>), grid, dim3(kMaxFolds * 256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 3) {
    hipLaunchKernelGGL((col_kernel_folds<double, 256, 3>), grid, dim3(kMaxFolds * 256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace zk
