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

}  // namespace umbir
