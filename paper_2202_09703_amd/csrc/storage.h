// Element types of trace, fine-grid and tap storage (umbir_acq.storage) and
// the matrix-core products the dense kernels use with them.  Accumulation is
// FP32 in every mode.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace umbir {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef short short4v __attribute__((ext_vector_type(4)));

template <int ST>
struct Store;

template <>
struct Store<UMBIR_STORAGE_F32> {
  using T = float;
  static __device__ __forceinline__ float get(T v) { return v; }
  static __device__ __forceinline__ T put(float v) { return v; }
};

template <>
struct Store<UMBIR_STORAGE_F16> {
  using T = _Float16;
  static __device__ __forceinline__ float get(T v) { return float(v); }
  static __device__ __forceinline__ T put(float v) { return T(v); }
  // D += A B for 32 x 8 A and 8 x 32 B, four values per lane each
  static __device__ __forceinline__ floatx16 mfma(uint2 a, uint2 b, floatx16 c) {
    half4 av, bv;
    __builtin_memcpy(&av, &a, 8);
    __builtin_memcpy(&bv, &b, 8);
    return __builtin_amdgcn_mfma_f32_32x32x8f16(av, bv, c, 0, 0, 0);
  }
};

// bfloat16 as 16-bit words: the upper half of an FP32, rounded to nearest even.
template <>
struct Store<UMBIR_STORAGE_BF16> {
  using T = uint16_t;
  static __device__ __forceinline__ float get(T v) { return __uint_as_float(uint32_t(v) << 16); }
  static __device__ __forceinline__ T put(float v) {
    const uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u) return T((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf / nan
    return T((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  }
  static __device__ __forceinline__ floatx16 mfma(uint2 a, uint2 b, floatx16 c) {
    short4v av, bv;
    __builtin_memcpy(&av, &a, 8);
    __builtin_memcpy(&bv, &b, 8);
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, c, 0, 0, 0);
  }
};

inline size_t storage_bytes(int st) { return st == UMBIR_STORAGE_F32 ? 4 : 2; }

// FP32 products on the bf16 matrix cores.  An FP32 value f splits exactly into
// three bf16 pieces, f = f1 + f2 + f3: f1 is f rounded to bf16 (8 significant
// bits, to nearest), f2 the remainder rounded likewise, and f3 what is left,
// at most 8 significant bits (each remainder is exact in FP32), so |f2| <=
// 2^-8 |f| and |f3| <= 2^-16 |f|.  A product a b is the sum of the six piece
// products a_i b_j with i + j <= 4; the three left out amount to at most
// about 2^-23 |a b|.  A piece product (8 x 8 bits) is exact in FP32, and the
// matrix cores accumulate in FP32, as the FP32 products do.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

struct Pieces8 {
  uint4 p[3];  // pieces 1, 2, 3 of 8 values, two bf16 per word, the first value in the low half
};

// x and y rounded to bf16 (nearest even), x in the low half
__device__ __forceinline__ unsigned bf16_pair(float x, float y) {
  const f32x2 v = {x, y};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}

// the three pieces of x and y, packed in pairs
__device__ __forceinline__ void split_pair_bf16x3(float x, float y, unsigned& p1, unsigned& p2, unsigned& p3) {
  p1 = bf16_pair(x, y);
  const float rx = x - __uint_as_float(p1 << 16), ry = y - __uint_as_float(p1 & 0xffff0000u);
  p2 = bf16_pair(rx, ry);
  const float sx = rx - __uint_as_float(p2 << 16), sy = ry - __uint_as_float(p2 & 0xffff0000u);
  p3 = bf16_pair(sx, sy);
}

__device__ __forceinline__ Pieces8 split8_bf16x3(const float4& x, const float4& y) {
  Pieces8 s;
  split_pair_bf16x3(x.x, x.y, s.p[0].x, s.p[1].x, s.p[2].x);
  split_pair_bf16x3(x.z, x.w, s.p[0].y, s.p[1].y, s.p[2].y);
  split_pair_bf16x3(y.x, y.y, s.p[0].z, s.p[1].z, s.p[2].z);
  split_pair_bf16x3(y.z, y.w, s.p[0].w, s.p[1].w, s.p[2].w);
  return s;
}

// D += A B for 32 x 16 A and 16 x 32 B given as pieces (lane l: row / column
// l % 32, contraction indices 8 (l / 32) .. + 7), the small products first
__device__ __forceinline__ floatx16 mfma_bf16x3(const uint4 (&a)[3], const uint4 (&b)[3], floatx16 c) {
  auto v = [](const uint4& u) { return __builtin_bit_cast(bf16x8, u); };
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(v(a[2]), v(b[0]), c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(v(a[1]), v(b[1]), c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(v(a[0]), v(b[2]), c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(v(a[1]), v(b[0]), c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(v(a[0]), v(b[1]), c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(v(a[0]), v(b[0]), c, 0, 0, 0);
  return c;
}

}  // namespace umbir
