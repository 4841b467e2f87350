// Buffer-resource loads and stores shared by the kernels of libmgar.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

// Buffer-resource access (gfx9 family descriptor: raw, stride 0, range
// checked). A load whose byte offset lies beyond the range returns 0 and a
// store there is dropped, so neighbours outside the grid, halo slots, planes
// outside a z-range and threads past the grid need no branch: they just use
// an offset at or above ZOOB, and every load of a kernel stays in flight
// together. Offsets are 32-bit: the buffer kernels are used while every array
// of the grid stays below 2 GiB (grid_fits_buffers); larger grids take the
// pointer kernels.
constexpr unsigned ZOOB = 0x80000000u;

__device__ inline __amdgpu_buffer_rsrc_t zrsrc(const void* p, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename E>
__device__ inline E zbload(const __amdgpu_buffer_rsrc_t& r, unsigned off);
template <>
__device__ inline double zbload<double>(const __amdgpu_buffer_rsrc_t& r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <>
__device__ inline float zbload<float>(const __amdgpu_buffer_rsrc_t& r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ inline uint16_t zbload<uint16_t>(const __amdgpu_buffer_rsrc_t& r, unsigned off) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
}

typedef unsigned int zu32x2 __attribute__((ext_vector_type(2)));
__device__ inline void zbstore(double v, const __amdgpu_buffer_rsrc_t& r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(zu32x2, v), r, (int)off, 0, 0);
}
__device__ inline void zbstore(float v, const __amdgpu_buffer_rsrc_t& r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}
