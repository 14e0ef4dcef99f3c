// Buffer-resource access to one plane of a grid array (gfx950, raw buffers).
//
// The streaming kernels address a plane as a wave-uniform base plus a uniform row offset
// and a per-lane column offset.  With a buffer resource whose base is the plane start,
// every load and store takes the column byte offset from a VGPR and the row byte offset
// from an SGPR, so no 64-bit address arithmetic runs per access.  The resource's size
// field is the plane's byte count: an access outside the plane reads 0 / is dropped
// instead of touching other memory.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace mgk {

// Data-format word of a raw 32-bit buffer resource on the gfx9 family.
constexpr int kBufferWord3 = 0x00020000;

typedef unsigned int BufU32x2 __attribute__((__vector_size__(8)));
typedef unsigned int BufU32x4 __attribute__((__vector_size__(16)));

struct PlaneBuf {
  __amdgpu_buffer_rsrc_t r;
};

template <typename T>
__device__ __forceinline__ PlaneBuf plane_buf(const T* array, size_t plane_bytes_offset,
                                              uint32_t plane_bytes)
{
  return PlaneBuf{__builtin_amdgcn_make_buffer_rsrc(
      const_cast<char*>(reinterpret_cast<const char*>(array) + plane_bytes_offset), 0,
      (int)plane_bytes, kBufferWord3)};
}

template <typename T>
__device__ __forceinline__ T buf_load(PlaneBuf b, uint32_t lane_off, uint32_t row_off);

template <>
__device__ __forceinline__ double buf_load<double>(PlaneBuf b, uint32_t lane_off, uint32_t row_off)
{
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)lane_off,
                                                                          (int)row_off, 0));
}

template <>
__device__ __forceinline__ float buf_load<float>(PlaneBuf b, uint32_t lane_off, uint32_t row_off)
{
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, (int)lane_off,
                                                                        (int)row_off, 0));
}

__device__ __forceinline__ void buf_store(double v, PlaneBuf b, uint32_t lane_off, uint32_t row_off)
{
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufU32x2, v), b.r,
                                        (int)lane_off, (int)row_off, 0);
}

__device__ __forceinline__ void buf_store(float v, PlaneBuf b, uint32_t lane_off, uint32_t row_off)
{
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), b.r, (int)lane_off,
                                        (int)row_off, 0);
}

// Two adjacent elements as one access (16 bytes for double, 8 for float).  The hardware
// needs only 4-byte alignment for these; the pair at an odd element index of a double array
// is 8-byte aligned.
__device__ __forceinline__ void buf_load2(PlaneBuf b, uint32_t lane_off, uint32_t row_off,
                                          double& a0, double& a1)
{
  const BufU32x4 v = __builtin_amdgcn_raw_buffer_load_b128(b.r, (int)lane_off, (int)row_off, 0);
  a0 = __hiloint2double((int)v[1], (int)v[0]);
  a1 = __hiloint2double((int)v[3], (int)v[2]);
}

__device__ __forceinline__ void buf_load2(PlaneBuf b, uint32_t lane_off, uint32_t row_off,
                                          float& a0, float& a1)
{
  const BufU32x2 v = __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)lane_off, (int)row_off, 0);
  a0 = __uint_as_float(v[0]);
  a1 = __uint_as_float(v[1]);
}

__device__ __forceinline__ void buf_store2(double a0, double a1, PlaneBuf b, uint32_t lane_off,
                                           uint32_t row_off)
{
  BufU32x4 v;
  v[0] = (unsigned)__double2loint(a0);
  v[1] = (unsigned)__double2hiint(a0);
  v[2] = (unsigned)__double2loint(a1);
  v[3] = (unsigned)__double2hiint(a1);
  __builtin_amdgcn_raw_buffer_store_b128(v, b.r, (int)lane_off, (int)row_off, 0);
}

__device__ __forceinline__ void buf_store2(float a0, float a1, PlaneBuf b, uint32_t lane_off,
                                           uint32_t row_off)
{
  BufU32x2 v;
  v[0] = __float_as_uint(a0);
  v[1] = __float_as_uint(a1);
  __builtin_amdgcn_raw_buffer_store_b64(v, b.r, (int)lane_off, (int)row_off, 0);
}

}  // namespace mgk
