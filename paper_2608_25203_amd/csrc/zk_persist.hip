// zk_persist.hip -- the persistent batch kernel (see zk_persist.hpp).
#include "zk_persist.hpp"

namespace zk {

namespace {

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename Tp>
__device__ __forceinline__ const Tp *uni_ptr(const Tp *p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return reinterpret_cast<const Tp *>(((unsigned long long)hi << 32) | lo);
}

// One block of a unit: the row or column body of its team shape, reading its
// LDS from the kernel's dynamic region.  Each shape's body is a function of
// its own, so the kernel needs the registers of its largest body rather than
// of all of them at once; the block-uniform arguments are made scalar again
// (readfirstlane) and the argument record is read into scalar registers.
template <typename real, int T, int E>
__device__ __noinline__ void prow(const RowArgs<real> *rargs, int rec, int index, int blk) {
  const RowArgs<real> a = uniform_load(uni_ptr(rargs) + uni(rec));
  row_body<real, T, E, true, kPBlock>(a, uni(index), uni(blk), nullptr);
}
template <typename real, int T, int E>
__device__ __noinline__ void pcol(const ColArgs<real> *cargs, int rec, int index, int blk) {
  const ColArgs<real> a = uniform_load(uni_ptr(cargs) + uni(rec));
  col_body<real, T, E, false, 1, true, kPBlock>(a, uni(index), uni(blk), nullptr);
}
template <typename real>
__device__ __forceinline__ void run_block(int shape, const RowArgs<real> *rargs, const ColArgs<real> *cargs, int rec,
                                          int index, int blk) {
  switch (shape) {
    case 0: prow<real, 64, 3>(rargs, rec, index, blk); break;
    case 1: prow<real, 64, 2>(rargs, rec, index, blk); break;
    case 2: prow<real, 128, 3>(rargs, rec, index, blk); break;
    case 3: prow<real, 128, 2>(rargs, rec, index, blk); break;
    case 4: prow<real, 256, 3>(rargs, rec, index, blk); break;
    case 5: prow<real, 256, 2>(rargs, rec, index, blk); break;
    case 6: prow<real, 512, 3>(rargs, rec, index, blk); break;
    case 7: prow<real, 512, 2>(rargs, rec, index, blk); break;
    case 8: pcol<real, 64, 3>(cargs, rec, index, blk); break;
    case 9: pcol<real, 64, 2>(cargs, rec, index, blk); break;
    case 10: pcol<real, 128, 3>(cargs, rec, index, blk); break;
    case 11: pcol<real, 128, 2>(cargs, rec, index, blk); break;
    case 12: pcol<real, 256, 3>(cargs, rec, index, blk); break;
    case 13: pcol<real, 256, 2>(cargs, rec, index, blk); break;
    case 14: pcol<real, 512, 3>(cargs, rec, index, blk); break;
    case 15: pcol<real, 512, 2>(cargs, rec, index, blk); break;
    default: break;
  }
}

// FP32: at most 128 VGPRs, so two workers fit a CU (the shapes' bodies need
// up to ~100 each; the rest is a small spill of the call stack); FP64 bodies
// need more, and one worker per CU is what fits.
template <typename real>
__global__ __launch_bounds__(kPBlock) __attribute__((amdgpu_waves_per_eu(sizeof(real) == 4 ? 4 : 2))) void persistent_kernel(const RowArgs<real> *__restrict__ rargs,
                                                         const ColArgs<real> *__restrict__ cargs,
                                                         const PUnit *__restrict__ units, int nunits,
                                                         uint32_t *ctr, uint32_t spin_limit) {
  __shared__ int s_unit, s_ok;
  for (;;) {
    __syncthreads();  // the previous unit's LDS and s_unit readers are done
    if (threadIdx.x == 0) {
      const int u = (int)atomicAdd(&ctr[0], 1u);
      int ok = 1;
      if (u < nunits) {
        const int tile = units[u].tile;
        const uint32_t need = units[u].need;
        uint32_t spins = 0;
        // poll with relaxed loads; one acquire fence once the count is seen
        // makes the tile's earlier units' results visible to this block
        while (__hip_atomic_load(&ctr[kCtrDone + tile], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (++spins > spin_limit) {
            atomicOr(&ctr[1], 1u);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(4);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      s_unit = u;
      s_ok = ok;
    }
    __syncthreads();
    const int u = s_unit;
    if (u >= nunits) return;  // uniform: every unit is taken
    const PUnit w = units[u];
    if (s_ok) {
      const int rec = w.rec;
      for (int b = 0; b < w.nblk; ++b) {
        __syncthreads();  // LDS of the previous block is free
        run_block<real>(w.shape, rargs, cargs, rec, w.index, w.blk0 + b);
      }
    }
    // Every wave's stores have reached the cache before the block counts the
    // unit; the release fence then makes them visible device-wide before the
    // count (the waiting side acquires on the count).
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(&ctr[kCtrDone + w.tile], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ void persist_reset_kernel(uint32_t *ctr, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) ctr[0] = 0u;
  if (i < n) ctr[kCtrDone + i] = 0u;
}
__global__ void persist_clear_flag_kernel(uint32_t *ctr) {
  if (threadIdx.x == 0) ctr[1] = 0u;
}

template <typename real>
int lds_bytes_of(int shape) {
  switch (shape % kPShapes) {
    case 0: return BodyLds<real, 64, 3, kPBlock>::bytes();
    case 1: return BodyLds<real, 64, 2, kPBlock>::bytes();
    case 2: return BodyLds<real, 128, 3, kPBlock>::bytes();
    case 3: return BodyLds<real, 128, 2, kPBlock>::bytes();
    case 4: return BodyLds<real, 256, 3, kPBlock>::bytes();
    case 5: return BodyLds<real, 256, 2, kPBlock>::bytes();
    case 6: return BodyLds<real, 512, 3, kPBlock>::bytes();
    case 7: return BodyLds<real, 512, 2, kPBlock>::bytes();
    default: return 0;
  }
}

// Dynamic LDS beyond the default limit must be allowed per kernel.
template <typename real>
hipError_t allow_lds(int lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(persistent_kernel<real>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

// Resident workers per CU: the runtime's occupancy answer, else the smaller
// of the register and LDS limits (512 VGPRs per SIMD lane in granules of 8,
// 4 SIMDs, 160 KiB of LDS per CU).
template <typename real>
int blocks_per_cu(int lds) {
  int n = 0;
  if (allow_lds<real>(lds) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persistent_kernel<real>, kPBlock, (size_t)lds) == hipSuccess &&
      n > 0)
    return n;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(persistent_kernel<real>)) != hipSuccess) return 0;
  const int regs = ((fa.numRegs > 0 ? fa.numRegs : 256) + 7) / 8 * 8;
  const int waves_per_simd = 512 / regs;
  const int by_regs = waves_per_simd * 4 / (kPBlock / 64);
  const int by_lds = (160 * 1024) / (lds + (int)fa.sharedSizeBytes + 1);
  return by_regs < by_lds ? by_regs : by_lds;
}

template <typename real>
hipError_t launch(int workers, int lds, hipStream_t s, const RowArgs<real> *rargs, const ColArgs<real> *cargs,
                  const PUnit *units, int nunits, uint32_t *ctr, uint32_t spin_limit) {
  const hipError_t e = allow_lds<real>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(persistent_kernel<real>, dim3(workers), dim3(kPBlock), (size_t)lds, s, rargs, cargs, units, nunits,
                     ctr, spin_limit);
  return hipGetLastError();
}

}  // namespace

template <>
int persist_lds_bytes<double>(int shape) { return lds_bytes_of<double>(shape); }
template <>
int persist_lds_bytes<float>(int shape) { return lds_bytes_of<float>(shape); }
template <>
int persistent_blocks_per_cu<double>(int lds) { return blocks_per_cu<double>(lds); }
template <>
int persistent_blocks_per_cu<float>(int lds) { return blocks_per_cu<float>(lds); }

template <>
hipError_t launch_persistent<double>(int workers, int lds, hipStream_t s, const RowArgs<double> *rargs,
                                     const ColArgs<double> *cargs, const PUnit *units, int nunits, uint32_t *ctr,
                                     uint32_t spin_limit) {
  return launch<double>(workers, lds, s, rargs, cargs, units, nunits, ctr, spin_limit);
}
template <>
hipError_t launch_persistent<float>(int workers, int lds, hipStream_t s, const RowArgs<float> *rargs,
                                    const ColArgs<float> *cargs, const PUnit *units, int nunits, uint32_t *ctr,
                                    uint32_t spin_limit) {
  return launch<float>(workers, lds, s, rargs, cargs, units, nunits, ctr, spin_limit);
}

hipError_t launch_persist_reset(uint32_t *ctr, int ntiles, hipStream_t s) {
  const int n = ntiles > 1 ? ntiles : 1;
  hipLaunchKernelGGL(persist_reset_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ctr, n);
  return hipGetLastError();
}
hipError_t launch_persist_clear_flag(uint32_t *ctr, hipStream_t s) {
  hipLaunchKernelGGL(persist_clear_flag_kernel, dim3(1), dim3(64), 0, s, ctr);
  return hipGetLastError();
}

}  // namespace zk
