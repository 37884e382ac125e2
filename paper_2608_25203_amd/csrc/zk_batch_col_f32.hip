// zk_batch_col_f32.hip -- batched col-pass kernel instances (float transforms);
// written by gen_batch_units.py.
#include "zk_kernels.hpp"

namespace zk {

template <>
const void *batch_col_kernel<float>(int T, int E) {
  if (T == 32 && E == 2) return reinterpret_cast<const void *>(&col_kernel_batch<float, 32, 2>);
  if (T == 32 && E == 3) return reinterpret_cast<const void *>(&col_kernel_batch<float, 32, 3>);
  if (T == 32 && E == 4) return reinterpret_cast<const void *>(&col_kernel_batch<float, 32, 4>);
  if (T == 32 && E == 6) return reinterpret_cast<const void *>(&col_kernel_batch<float, 32, 6>);
  if (T == 32 && E == 8) return reinterpret_cast<const void *>(&col_kernel_batch<float, 32, 8>);
  if (T == 32 && E == 12) return reinterpret_cast<const void *>(&col_kernel_batch<float, 32, 12>);
  if (T == 64 && E == 2) return reinterpret_cast<const void *>(&col_kernel_batch<float, 64, 2>);
  if (T == 64 && E == 3) return reinterpret_cast<const void *>(&col_kernel_batch<float, 64, 3>);
  if (T == 64 && E == 4) return reinterpret_cast<const void *>(&col_kernel_batch<float, 64, 4>);
  if (T == 64 && E == 6) return reinterpret_cast<const void *>(&col_kernel_batch<float, 64, 6>);
  if (T == 64 && E == 8) return reinterpret_cast<const void *>(&col_kernel_batch<float, 64, 8>);
  if (T == 64 && E == 12) return reinterpret_cast<const void *>(&col_kernel_batch<float, 64, 12>);
  if (T == 128 && E == 2) return reinterpret_cast<const void *>(&col_kernel_batch<float, 128, 2>);
  if (T == 128 && E == 3) return reinterpret_cast<const void *>(&col_kernel_batch<float, 128, 3>);
  if (T == 128 && E == 4) return reinterpret_cast<const void *>(&col_kernel_batch<float, 128, 4>);
  if (T == 128 && E == 6) return reinterpret_cast<const void *>(&col_kernel_batch<float, 128, 6>);
  if (T == 128 && E == 8) return reinterpret_cast<const void *>(&col_kernel_batch<float, 128, 8>);
  if (T == 128 && E == 12) return reinterpret_cast<const void *>(&col_kernel_batch<float, 128, 12>);
  if (T == 256 && E == 2) return reinterpret_cast<const void *>(&col_kernel_batch<float, 256, 2>);
  if (T == 256 && E == 3) return reinterpret_cast<const void *>(&col_kernel_batch<float, 256, 3>);
  if (T == 256 && E == 4) return reinterpret_cast<const void *>(&col_kernel_batch<float, 256, 4>);
  if (T == 256 && E == 6) return reinterpret_cast<const void *>(&col_kernel_batch<float, 256, 6>);
  if (T == 256 && E == 8) return reinterpret_cast<const void *>(&col_kernel_batch<float, 256, 8>);
  if (T == 256 && E == 12) return reinterpret_cast<const void *>(&col_kernel_batch<float, 256, 12>);
  if (T == 512 && E == 2) return reinterpret_cast<const void *>(&col_kernel_batch<float, 512, 2>);
  if (T == 512 && E == 3) return reinterpret_cast<const void *>(&col_kernel_batch<float, 512, 3>);
  if (T == 512 && E == 4) return reinterpret_cast<const void *>(&col_kernel_batch<float, 512, 4>);
  if (T == 512 && E == 6) return reinterpret_cast<const void *>(&col_kernel_batch<float, 512, 6>);
  if (T == 1024 && E == 2) return reinterpret_cast<const void *>(&col_kernel_batch<float, 1024, 2>);
  if (T == 1024 && E == 3) return reinterpret_cast<const void *>(&col_kernel_batch<float, 1024, 3>);
  return nullptr;
}

template <>
hipError_t launch_batch_col<float>(int T, int E, dim3 grid, hipStream_t s, const ColArgs<float> *args,
                                   const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph) {
  if (T == 32 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 32, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 3) {
    hipLaunchKernelGGL((col_kernel_batch<float, 32, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<float, 32, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<float, 32, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<float, 32, 8>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 12) {
    hipLaunchKernelGGL((col_kernel_batch<float, 32, 12>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 64, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 3) {
    hipLaunchKernelGGL((col_kernel_batch<float, 64, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<float, 64, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<float, 64, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<float, 64, 8>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 12) {
    hipLaunchKernelGGL((col_kernel_batch<float, 64, 12>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 128, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 3) {
    hipLaunchKernelGGL((col_kernel_batch<float, 128, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<float, 128, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<float, 128, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<float, 128, 8>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 12) {
    hipLaunchKernelGGL((col_kernel_batch<float, 128, 12>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 256, 2>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 3) {
    hipLaunchKernelGGL((col_kernel_batch<float, 256, 3>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<float, 256, 4>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<float, 256, 6>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<float, 256, 8>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 12) {
    hipLaunchKernelGGL((col_kernel_batch<float, 256, 12>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 512, 2>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 3) {
    hipLaunchKernelGGL((col_kernel_batch<float, 512, 3>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<float, 512, 4>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 6) {
    hipLaunchKernelGGL((col_kernel_batch<float, 512, 6>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 1024 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 1024, 2>), grid, dim3(1024), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 1024 && E == 3) {
    hipLaunchKernelGGL((col_kernel_batch<float, 1024, 3>), grid, dim3(1024), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_batch_col_lift<float>(int T, int E, dim3 grid, hipStream_t s, const ColArgs<float> *args,
                                        const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph) {
  if (T == 32 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 32, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<float, 32, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 32 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<float, 32, 8, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 64, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<float, 64, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<float, 64, 8, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 128, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<float, 128, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<float, 128, 8, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 256, 2, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<float, 256, 4, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 8) {
    hipLaunchKernelGGL((col_kernel_batch<float, 256, 8, true>), grid, dim3(256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 512, 2, true>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 512 && E == 4) {
    hipLaunchKernelGGL((col_kernel_batch<float, 512, 4, true>), grid, dim3(512), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 1024 && E == 2) {
    hipLaunchKernelGGL((col_kernel_batch<float, 1024, 2, true>), grid, dim3(1024), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_batch_col_folds<float>(int T, int E, dim3 grid, hipStream_t s, const ColArgs<float> *args,
                                         const BatchItem *items, int tile0, int first0, const void *sched0, PhysArgs ph) {
  if (T == 64 && E == 2) {
    hipLaunchKernelGGL((col_kernel_folds<float, 64, 2>), grid, dim3(kMaxFolds * 64), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 64 && E == 3) {
    hipLaunchKernelGGL((col_kernel_folds<float, 64, 3>), grid, dim3(kMaxFolds * 64), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 2) {
    hipLaunchKernelGGL((col_kernel_folds<float, 128, 2>), grid, dim3(kMaxFolds * 128), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 128 && E == 3) {
    hipLaunchKernelGGL((col_kernel_folds<float, 128, 3>), grid, dim3(kMaxFolds * 128), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 2) {
    hipLaunchKernelGGL((col_kernel_folds<float, 256, 2>), grid, dim3(kMaxFolds * 256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  if (T == 256 && E == 3) {
    hipLaunchKernelGGL((col_kernel_folds<float, 256, 3>), grid, dim3(kMaxFolds * 256), 0, s, args, items, tile0, first0, sched0, ph);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace zk
