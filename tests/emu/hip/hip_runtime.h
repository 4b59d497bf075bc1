// Host stand-in for <hip/hip_runtime.h>: the subset of HIP the library uses,
// mapped onto the emulator of emu_runtime.h (test infrastructure only; see
// tests/test_kernel_emu.py).  Device code: the kernel qualifiers, thread
// indices, barriers and cross-lane builtins.  Host API: device memory is
// host memory from a registry of allocations (so that pointer checks see
// "device" memory), copies are synchronous, streams are tokens, events read
// the host clock, and the one device reports gfx950.
#pragma once
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <map>
#include <mutex>

#include "../emu_runtime.h"

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) alignas(n)

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
  ::emu::mfma<std::decay_t<decltype(c)>, double, true>((a), (b), (c))
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) \
  ::emu::mfma<std::decay_t<decltype(c)>, float, false>((a), (b), (c))
#define __shfl(...) ::emu::shfl(__VA_ARGS__)
#define __shfl_xor(...) ::emu::shfl_xor(__VA_ARGS__)
#define __shfl_up(...) ::emu::shfl_up(__VA_ARGS__)
#define __ballot(p) ::emu::ballot((p))
#define __ffsll(x) __builtin_ffsll((long long)(x))
#define __popcll(x) __builtin_popcountll((unsigned long long)(x))

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

// ---- host API ---------------------------------------------------------------
typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotReady = 600
} hipError_t;
typedef struct ihipStream_t* hipStream_t;
struct EmuEvent { std::chrono::steady_clock::time_point t; };
typedef EmuEvent* hipEvent_t;
typedef enum hipFuncAttribute {
  hipFuncAttributeMaxDynamicSharedMemorySize = 8
} hipFuncAttribute;
typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;
typedef enum hipMemoryType {
  hipMemoryTypeUnregistered = 0,
  hipMemoryTypeHost = 1,
  hipMemoryTypeDevice = 2,
  hipMemoryTypeManaged = 3
} hipMemoryType;
struct hipPointerAttribute_t {
  hipMemoryType type;
  int device;
  void* devicePointer;
  void* hostPointer;
  int isManaged;
  unsigned allocationFlags;
};
struct hipDeviceProp_t {
  char name[256];
  char gcnArchName[256];
  size_t totalGlobalMem;
  int multiProcessorCount;
};
#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u
#define hipHostMallocDefault 0u
#define HIP_SYMBOL(x) ((const void*)&(x))

namespace emu {
// "device" allocations: start -> size
inline std::map<uintptr_t, size_t>& registry() {
  static std::map<uintptr_t, size_t> r;
  return r;
}
inline std::mutex& registry_mu() {
  static std::mutex m;
  return m;
}
inline bool is_device(const void* p) {
  std::lock_guard<std::mutex> g(registry_mu());
  auto& r = registry();
  auto it = r.upper_bound(reinterpret_cast<uintptr_t>(p));
  if (it == r.begin()) return false;
  --it;
  return reinterpret_cast<uintptr_t>(p) < it->first + it->second;
}
inline void* device_alloc(size_t n) {
  void* p = std::malloc(n ? n : 1);
  if (!p) return nullptr;
  std::memset(p, 0xFF, n);   // device memory starts undefined: NaN / -1
  std::lock_guard<std::mutex> g(registry_mu());
  registry()[reinterpret_cast<uintptr_t>(p)] = n ? n : 1;
  return p;
}
inline void register_device(const void* p, size_t n) {
  std::lock_guard<std::mutex> g(registry_mu());
  registry()[reinterpret_cast<uintptr_t>(p)] = n;
}
inline bool device_free(void* p) {
  {
    std::lock_guard<std::mutex> g(registry_mu());
    auto it = registry().find(reinterpret_cast<uintptr_t>(p));
    if (it == registry().end()) return false;
    registry().erase(it);
  }
  std::free(p);
  return true;
}
}  // namespace emu

inline hipError_t hipMalloc(void** p, size_t n) {
  *p = ::emu::device_alloc(n);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
template <class T>
inline hipError_t hipMalloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), n);
}
inline hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  return ::emu::device_free(p) ? hipSuccess : hipErrorInvalidValue;
}
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned = 0) {
  *p = std::malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
template <class T>
inline hipError_t hipHostMalloc(T** p, size_t n, unsigned f = 0) {
  return hipHostMalloc(reinterpret_cast<void**>(p), n, f);
}
inline hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  if (n) std::memmove(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n,
                                 hipMemcpyKind k, hipStream_t = nullptr) {
  return hipMemcpy(d, s, n, k);
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  static char token;
  *s = reinterpret_cast<hipStream_t>(&token);
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new EmuEvent{std::chrono::steady_clock::now()};
  return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  return hipEventCreate(e);
}
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t = nullptr) {
  e->t = std::chrono::steady_clock::now();
  return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
  return hipSuccess;
}
inline hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
inline hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipSetDevice(int d) {
  return d == 0 ? hipSuccess : hipErrorInvalidValue;
}
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d) {
  if (d != 0) return hipErrorInvalidValue;
  std::memset(p, 0, sizeof *p);
  std::strcpy(p->name, "host emulation");
  std::strcpy(p->gcnArchName, "gfx950");
  p->totalGlobalMem = size_t(32) << 30;
  p->multiProcessorCount = 256;
  return hipSuccess;
}
inline hipError_t hipMemGetInfo(size_t* free_b, size_t* total_b) {
  *total_b = size_t(32) << 30;
  *free_b = size_t(16) << 30;
  return hipSuccess;
}
inline hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a,
                                          const void* p) {
  std::memset(a, 0, sizeof *a);
  if (!::emu::is_device(p)) return hipErrorInvalidValue;
  a->type = hipMemoryTypeDevice;
  a->device = 0;
  a->devicePointer = const_cast<void*>(p);
  return hipSuccess;
}
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
inline hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) {
  return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t e) {
  return e == hipSuccess ? "hipSuccess" : "hip error (emulated)";
}
#define hipLaunchKernelGGL(kern, grid, block, lds, stream, ...) \
  ::emu::launch((kern), dim3(grid), dim3(block), (size_t)(lds), __VA_ARGS__)
