// Complex helpers for the kernels: float2 / double2 / packed bf16 pairs.
#pragma once

#include <hip/hip_runtime.h>

namespace tb {

template <class T>
struct CplxOf;
template <>
struct CplxOf<double> {
  using type = double2;
};
template <>
struct CplxOf<float> {
  using type = float2;
};

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class C>
__device__ __forceinline__ C czero() {
  C z;
  z.x = 0;
  z.y = 0;
  return z;
}

// acc + a * b
template <class C>
__device__ __forceinline__ C cfma(C acc, C a, C b) {
  acc.x = fmaT(a.x, b.x, acc.x);
  acc.x = fmaT(-a.y, b.y, acc.x);
  acc.y = fmaT(a.x, b.y, acc.y);
  acc.y = fmaT(a.y, b.x, acc.y);
  return acc;
}

// acc + conj(a) * b
template <class C>
__device__ __forceinline__ C cfma_conj(C acc, C a, C b) {
  acc.x = fmaT(a.x, b.x, acc.x);
  acc.x = fmaT(a.y, b.y, acc.x);
  acc.y = fmaT(a.x, b.y, acc.y);
  acc.y = fmaT(-a.y, b.x, acc.y);
  return acc;
}

template <class C>
__device__ __forceinline__ C cadd(C a, C b) {
  a.x += b.x;
  a.y += b.y;
  return a;
}

template <class C>
__device__ __forceinline__ C cconj(C a) {
  a.y = -a.y;
  return a;
}

// bf16 <-> fp32 (round to nearest even on the way down)
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}

__host__ __device__ inline unsigned short f32_to_bf16(float f) {
  unsigned u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  unsigned lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (unsigned short)(u >> 16);
}

}  // namespace tb
