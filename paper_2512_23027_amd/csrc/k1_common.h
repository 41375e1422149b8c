// Device helpers shared by the hand-written kernels (kernels.hip) and the
// generated SG-apply kernels (k1_gen_*.hip): raw buffer loads and stores and
// the XCD-aware workgroup mapping.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace sgw {
namespace k {

// Raw buffer access: 128-bit resource (base address, no stride, no range
// limit) with a per-lane 32-bit byte offset and a wave-uniform byte offset.
typedef unsigned int sgw_u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)0xffffffffu,
                                           0x00020000);
}
template <typename T> __device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <> __device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <> __device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ int buf_load<int>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}
template <typename T> __device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, int voff, int soff);
template <> __device__ __forceinline__ void buf_store<double>(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(sgw_u32x2, v), r, voff, soff, 0);
}
template <> __device__ __forceinline__ void buf_store<float>(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
}

// A zero the compiler cannot see through (a scalar register set by an asm
// statement): added to a load offset, it makes otherwise identical loads of
// different program points distinct.
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
}

// Byte offset of the per-wave p'q partials in the LDS of a shared PCG kernel:
// after the larger of the staged halo (hmax entries of eb bytes) and the
// wave partials of one output slice (rb bytes), 8-byte aligned.
__host__ __device__ inline size_t shared_pq_offset(size_t hmax, size_t eb, size_t rb) {
  const size_t a = hmax * eb;
  return ((a > rb ? a : rb) + 7) & ~(size_t)7;
}

// Kernels with the Galerkin tensor of a fixed basis unrolled (gen_k1.py).
// Workgroups are dispatched round-robin over the 8 XCDs (workgroup i to XCD
// i % 8), each with its own L2.  This bijection gives XCD x a contiguous
// range of logical indices, so neighbouring row groups, whose column halos
// overlap, share an L2.
__device__ __forceinline__ int xcd_group(int i, int n) {
  const int nx = 8, x = i % nx, k = i / nx;
  const int per = n / nx, rem = n % nx;
  return x * per + min(x, rem) + k;
}

}  // namespace k
}  // namespace sgw
