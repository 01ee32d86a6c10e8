// Wavefront helpers shared by the libbfs kernels (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bfsmi {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Number of set bits of `m` below the calling lane.
__device__ __forceinline__ unsigned lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__device__ __forceinline__ unsigned long long wave_or(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o);
  return x;
}

// The global-memory view of a device pointer whose address space the
// compiler cannot see (one loaded from memory, such as the output arrays in
// the control block).  Accesses through a plain pointer of that kind become
// flat instructions, which also count as LDS operations, so every later wait
// for an LDS access would wait for them too; through this view they are
// global loads and stores.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gptr(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

// Loads and stores of data that workgroups hand to each other within one
// kernel: with `coherent`, agent-scope atomic accesses, which are performed
// at the device-wide coherence point (an XCD's L2 is not coherent with the
// others'), so no cache write-back or invalidation is needed; otherwise plain
// accesses (a kernel boundary orders them).
template <class T>
__device__ __forceinline__ T ld_x(const T *p, bool coherent) {
  return coherent ? __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *p;
}
template <class T>
__device__ __forceinline__ void st_x(T *p, T v, bool coherent) {
  if (coherent)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}

// Workgroup order that gives each XCD a contiguous range of workgroups
// (consecutive workgroup ids are dealt round-robin to the 8 XCDs).
__device__ __forceinline__ int64_t xcd_block(int64_t nblocks) {
  constexpr int kXcd = 8;
  const int64_t b = blockIdx.x;
  const int64_t per = nblocks / kXcd;
  if (per == 0 || b >= per * kXcd) return b;
  return (b % kXcd) * per + b / kXcd;
}

}  // namespace bfsmi
