// Device-side helpers shared by the grouped-GEMM and split-plane kernels.
#pragma once
#include "internal.h"

namespace bsd {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// tagged pointer -> address (bits 56..63 select the base)
__device__ __forceinline__ const double* resolve(uint64_t t, const GBases& b) {
  return reinterpret_cast<const double*>(b.b[t >> kTagShift] + (t & ((1ull << kTagShift) - 1)));
}

// float -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ double bf16_to_double(unsigned short h) {
  return (double)__uint_as_float(((unsigned int)h) << 16);
}

// wave-uniform copies (values every lane of the wave already agrees on)
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni64(int64_t x) {
  const uint64_t u = (uint64_t)x;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double unid(double x) {
  return __longlong_as_double(uni64(__double_as_longlong(x)));
}

}  // namespace bsd
