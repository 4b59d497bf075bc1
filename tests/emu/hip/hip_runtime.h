// Host stand-in for <hip/hip_runtime.h>: the subset of HIP the library's
// kernels and their launch code use, mapped onto the emulator of
// emu_runtime.h (test infrastructure only; see tests/test_kernel_emu.py).
#pragma once
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../emu_runtime.h"

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static

#define threadIdx (::emu::cur()->tidx)
#define blockIdx (::emu::blk()->bidx)
#define blockDim (::emu::blk()->bdim)
#define gridDim (::emu::blk()->gdim)
#define warpSize 64

#define __syncthreads() ::emu::syncthreads()
#define __builtin_amdgcn_wave_barrier() ::emu::wave_barrier()
#define __builtin_amdgcn_fence(order, scope) ((void)0)
#define __builtin_amdgcn_sched_barrier(mask) ((void)0)
#define __builtin_amdgcn_s_setprio(p) ((void)0)
#define __builtin_amdgcn_readlane(v, l) ::emu::readlane((v), (l))
#define __builtin_amdgcn_readfirstlane(v) ::emu::readfirstlane((v))
#define __builtin_amdgcn_update_dpp ::emu::update_dpp
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) \
  ::emu::mfma<decltype(c), double, true>((a), (b), (c))
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) \
  ::emu::mfma<decltype(c), float, false>((a), (b), (c))
#define __shfl(...) ::emu::shfl(__VA_ARGS__)
#define __shfl_xor(...) ::emu::shfl_xor(__VA_ARGS__)
#define __shfl_up(...) ::emu::shfl_up(__VA_ARGS__)
#define __ballot(p) ::emu::ballot((p))
#define __ffsll(x) __builtin_ffsll((long long)(x))

inline long long __double_as_longlong(double d) {
  long long v;
  memcpy(&v, &d, sizeof v);
  return v;
}
inline double __longlong_as_double(long long v) {
  double d;
  memcpy(&d, &v, sizeof d);
  return d;
}
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }

// host API
typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2
} hipError_t;
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef enum hipFuncAttribute {
  hipFuncAttributeMaxDynamicSharedMemorySize = 8
} hipFuncAttribute;
inline hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) {
  return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
#define hipLaunchKernelGGL(kern, grid, block, lds, stream, ...) \
  ::emu::launch((kern), dim3(grid), dim3(block), (size_t)(lds), __VA_ARGS__)
