// Element access helpers for the dense operands: FP32 or BF16 storage, FP32 arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spmm {

struct F32E {
  using T = float;
};
struct BF16E {
  using T = uint16_t;
};

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// FP32 -> BF16 with round-to-nearest-even on the bit pattern: adding 0x7FFF plus
// the lowest kept bit carries into the kept half exactly when the discarded half
// is above the midpoint, or at it with an odd kept half.  NaN maps to 0x7FC0.
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0u;
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// Load V consecutive elements starting at p (aligned to V elements) as FP32.
template <typename E, int V>
__device__ __forceinline__ void load_vec(const typename E::T* p, float (&x)[V]) {
  if constexpr (sizeof(typename E::T) == 4) {
    if constexpr (V == 1) {
      x[0] = p[0];
    } else if constexpr (V == 2) {
      float2 a = *reinterpret_cast<const float2*>(p);
      x[0] = a.x; x[1] = a.y;
    } else if constexpr (V == 4) {
      float4 a = *reinterpret_cast<const float4*>(p);
      x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    } else {
      static_assert(V == 8, "fp32 vector width");
      float4 a = reinterpret_cast<const float4*>(p)[0];
      float4 b = reinterpret_cast<const float4*>(p)[1];
      x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
      x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
    }
  } else {
    if constexpr (V == 1) {
      x[0] = bf16_bits_to_f32(p[0]);
    } else if constexpr (V == 2) {
      uint32_t a = *reinterpret_cast<const uint32_t*>(p);
      x[0] = __uint_as_float(a << 16); x[1] = __uint_as_float(a & 0xFFFF0000u);
    } else if constexpr (V == 4) {
      uint2 a = *reinterpret_cast<const uint2*>(p);
      x[0] = __uint_as_float(a.x << 16); x[1] = __uint_as_float(a.x & 0xFFFF0000u);
      x[2] = __uint_as_float(a.y << 16); x[3] = __uint_as_float(a.y & 0xFFFF0000u);
    } else {
      static_assert(V == 8, "bf16 vector width");
      uint4 a = *reinterpret_cast<const uint4*>(p);
      x[0] = __uint_as_float(a.x << 16); x[1] = __uint_as_float(a.x & 0xFFFF0000u);
      x[2] = __uint_as_float(a.y << 16); x[3] = __uint_as_float(a.y & 0xFFFF0000u);
      x[4] = __uint_as_float(a.z << 16); x[5] = __uint_as_float(a.z & 0xFFFF0000u);
      x[6] = __uint_as_float(a.w << 16); x[7] = __uint_as_float(a.w & 0xFFFF0000u);
    }
  }
}

// The same load from an integer device address, marked as global memory so that
// the compiler emits global (not flat) loads.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
#define SPMM_GLOBAL(T) const __attribute__((address_space(1))) T*

template <typename E, int V>
__device__ __forceinline__ void load_vec_at(uint64_t addr, float (&x)[V]) {
  using T = typename E::T;
  if constexpr (sizeof(T) == 4) {
    if constexpr (V == 1) {
      x[0] = *(SPMM_GLOBAL(float))addr;
    } else if constexpr (V == 2) {
      const f32x2_t a = *(SPMM_GLOBAL(f32x2_t))addr;
      x[0] = a.x; x[1] = a.y;
    } else {
      static_assert(V == 4, "fp32 vector width");
      const f32x4_t a = *(SPMM_GLOBAL(f32x4_t))addr;
      x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    }
  } else {
    if constexpr (V == 1) {
      x[0] = bf16_bits_to_f32(*(SPMM_GLOBAL(uint16_t))addr);
    } else if constexpr (V == 2) {
      const uint32_t a = *(SPMM_GLOBAL(uint32_t))addr;
      x[0] = __uint_as_float(a << 16); x[1] = __uint_as_float(a & 0xFFFF0000u);
    } else if constexpr (V == 4) {
      const u32x2_t a = *(SPMM_GLOBAL(u32x2_t))addr;
      x[0] = __uint_as_float(a.x << 16); x[1] = __uint_as_float(a.x & 0xFFFF0000u);
      x[2] = __uint_as_float(a.y << 16); x[3] = __uint_as_float(a.y & 0xFFFF0000u);
    } else {
      static_assert(V == 8, "bf16 vector width");
      const u32x4_t a = *(SPMM_GLOBAL(u32x4_t))addr;
      x[0] = __uint_as_float(a.x << 16); x[1] = __uint_as_float(a.x & 0xFFFF0000u);
      x[2] = __uint_as_float(a.y << 16); x[3] = __uint_as_float(a.y & 0xFFFF0000u);
      x[4] = __uint_as_float(a.z << 16); x[5] = __uint_as_float(a.z & 0xFFFF0000u);
      x[6] = __uint_as_float(a.w << 16); x[7] = __uint_as_float(a.w & 0xFFFF0000u);
    }
  }
}
#undef SPMM_GLOBAL

// Store V FP32 values to V consecutive elements (rounded once for BF16).
template <typename E, int V>
__device__ __forceinline__ void store_vec(typename E::T* p, const float (&x)[V]) {
  if constexpr (sizeof(typename E::T) == 4) {
    if constexpr (V == 1) {
      p[0] = x[0];
    } else if constexpr (V == 2) {
      *reinterpret_cast<float2*>(p) = make_float2(x[0], x[1]);
    } else if constexpr (V == 4) {
      *reinterpret_cast<float4*>(p) = make_float4(x[0], x[1], x[2], x[3]);
    } else {
      reinterpret_cast<float4*>(p)[0] = make_float4(x[0], x[1], x[2], x[3]);
      reinterpret_cast<float4*>(p)[1] = make_float4(x[4], x[5], x[6], x[7]);
    }
  } else {
    uint32_t h[V];
#pragma unroll
    for (int e = 0; e < V; ++e) h[e] = f32_to_bf16_bits(x[e]);
    if constexpr (V == 1) {
      p[0] = (uint16_t)h[0];
    } else if constexpr (V == 2) {
      *reinterpret_cast<uint32_t*>(p) = h[0] | (h[1] << 16);
    } else if constexpr (V == 4) {
      *reinterpret_cast<uint2*>(p) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    } else {
      *reinterpret_cast<uint4*>(p) = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16),
                                                h[4] | (h[5] << 16), h[6] | (h[7] << 16));
    }
  }
}

// The same store with a non-temporal hint: output rows are written once and never
// re-read by the kernel, so they should not displace gathered B rows in the caches.
template <typename E, int V>
__device__ __forceinline__ void store_vec_nt(typename E::T* p, const float (&x)[V]) {
  if constexpr (sizeof(typename E::T) == 4) {
    if constexpr (V == 1) {
      __builtin_nontemporal_store(x[0], p);
    } else if constexpr (V == 2) {
      f32x2_t v = {x[0], x[1]};
      __builtin_nontemporal_store(v, reinterpret_cast<f32x2_t*>(p));
    } else if constexpr (V == 4) {
      f32x4_t v = {x[0], x[1], x[2], x[3]};
      __builtin_nontemporal_store(v, reinterpret_cast<f32x4_t*>(p));
    } else {
      f32x4_t v0 = {x[0], x[1], x[2], x[3]}, v1 = {x[4], x[5], x[6], x[7]};
      __builtin_nontemporal_store(v0, reinterpret_cast<f32x4_t*>(p));
      __builtin_nontemporal_store(v1, reinterpret_cast<f32x4_t*>(p) + 1);
    }
  } else {
    uint32_t h[V];
#pragma unroll
    for (int e = 0; e < V; ++e) h[e] = f32_to_bf16_bits(x[e]);
    if constexpr (V == 1) {
      __builtin_nontemporal_store((uint16_t)h[0], p);
    } else if constexpr (V == 2) {
      __builtin_nontemporal_store(h[0] | (h[1] << 16), reinterpret_cast<uint32_t*>(p));
    } else if constexpr (V == 4) {
      u32x2_t v = {h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
      __builtin_nontemporal_store(v, reinterpret_cast<u32x2_t*>(p));
    } else {
      u32x4_t v = {h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
      __builtin_nontemporal_store(v, reinterpret_cast<u32x4_t*>(p));
    }
  }
}

// FP32 partial sums (always FP32, V consecutive, aligned).
template <int V>
__device__ __forceinline__ void load_f32v(const float* p, float (&x)[V]) {
  load_vec<F32E, V>(p, x);
}
template <int V>
__device__ __forceinline__ void store_f32v(float* p, const float (&x)[V]) {
  store_vec<F32E, V>(p, x);
}

}  // namespace spmm
