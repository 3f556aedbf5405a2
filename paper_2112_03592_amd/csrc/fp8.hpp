// FP8 storage type of network activations (included by the kernels that
// take it: the child-map tree fill and the gather-path layers).
#pragma once

#include "common.hpp"

namespace apr {

// FP8 E4M3 in the OCP "FN" encoding: sign, 4 exponent bits (bias 7), 3
// mantissa bits; no infinities, 0x7f / 0xff are NaN, largest finite 448,
// subnormals down to 2^-9.  FP32 -> FP8 is written out on the bits: round to
// nearest even, finite values and infinities saturate to +-448.
struct fp8e4m3 {
  uint8_t bits;
};
// FP8 -> FP32 on the conversion unit (gfx950 reads E4M3 in the OCP encoding);
// four codes of a 32-bit word at a time in the vector loads.
template <> __device__ inline float to_f32<fp8e4m3>(fp8e4m3 v) {
  return __builtin_amdgcn_cvt_f32_fp8(int(v.bits), 0);
}
__device__ inline void fp8x4_to_f32(uint32_t c, float* f) {
  const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(int(c), false);
  const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(int(c), true);
  f[0] = lo[0];
  f[1] = lo[1];
  f[2] = hi[0];
  f[3] = hi[1];
}
template <>
__device__ inline void load_vec<fp8e4m3, 16>(const fp8e4m3* p, float* v) {
  const uint4 raw = *reinterpret_cast<const uint4*>(p);
  fp8x4_to_f32(raw.x, v);
  fp8x4_to_f32(raw.y, v + 4);
  fp8x4_to_f32(raw.z, v + 8);
  fp8x4_to_f32(raw.w, v + 12);
}
template <> __device__ inline fp8e4m3 from_f32<fp8e4m3>(float v) {
  const uint32_t b = __float_as_uint(v);
  const uint8_t sign = uint8_t((b >> 24) & 0x80u);
  const uint32_t a = b & 0x7fffffffu;
  if (a > 0x7f800000u) return fp8e4m3{uint8_t(sign | 0x7fu)};     // NaN
  if (a >= 0x43e80000u) return fp8e4m3{uint8_t(sign | 0x7eu)};    // |v| >= 464: saturate to 448
  if (a < 0x3c800000u)                                             // |v| < 2^-6: multiples of 2^-9
    return fp8e4m3{uint8_t(sign | uint8_t(rintf(__uint_as_float(a) * 512.f)))};
  const uint32_t r = a + 0x7ffffu + ((a >> 20) & 1u);              // nearest even on the 20 dropped bits
  return fp8e4m3{uint8_t(sign | (((r >> 23) - 120u) << 3) | ((r >> 20) & 7u))};
}

}  // namespace apr
