// Device-side rounding to the stored number formats (round to nearest even).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// OCP E4M3FN: round |v| (already scaled) to the nearest code, ties to even,
// saturating at 448 (code 0x7E).  Subnormals are multiples of 2^-9.
__device__ __forceinline__ uint8_t f32_to_e4m3_rne(float v) {
  const uint8_t sgn = v < 0.f ? 0x80 : 0;
  const float a = fabsf(v);
  if (!(a < 448.f)) return sgn | 0x7E;
  if (a < 0x1p-6f) {
    const int m = static_cast<int>(rintf(a * 512.f));   // m == 8 is the code of 2^-6
    return sgn | static_cast<uint8_t>(m);
  }
  int e = 0;
  const float f = frexpf(a, &e);   // a = f * 2^e, f in [0.5, 1)
  int E = e - 1;                   // a = (2f) * 2^E, 2f in [1, 2)
  int m = static_cast<int>(rintf((2.f * f - 1.f) * 8.f));
  if (m == 8) {
    m = 0;
    ++E;
  }
  int code = ((E + 7) << 3) | m;
  if (code > 0x7E) code = 0x7E;
  return sgn | static_cast<uint8_t>(code);
}
