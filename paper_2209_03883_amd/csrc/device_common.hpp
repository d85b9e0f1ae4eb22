// Device-side helpers shared by every radar kernel: complex arithmetic on
// float2 and the library's twiddle table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Twiddle table, one contiguous block per power-of-two length:
//   g_radar_tw[L + x] = W_L^x = exp(-2*pi*i*x/L),   L = 1, 2, 4, ..., RADAR_TW_LMAX,  0 <= x < L,
// each value computed on the host in double precision and rounded once to
// float.  Blocks are contiguous so that the entries one FFT stage touches sit
// together in cache.
#define RADAR_TW_LOG2 14
#define RADAR_TW_LMAX (1 << RADAR_TW_LOG2)
#define RADAR_TW_ENTRIES (2 * RADAR_TW_LMAX)

extern __device__ float2 g_radar_tw[RADAR_TW_ENTRIES];

namespace radar {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * b
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

// W_L^x = exp(-2*pi*i*x/L) for a power-of-two L <= RADAR_TW_LMAX and 0 <= x < L.
__device__ __forceinline__ float2 twiddle(int L, int x) { return g_radar_tw[L + x]; }

// Periodic window value w(i) of length L (a power of two):
// Hann 0.5 - 0.5 cos(2 pi i/L); Hamming 0.54 - 0.46 cos(2 pi i/L); rect 1.
__device__ __forceinline__ float window_value(int kind, int i, int L) {
  if (kind == 0) return 1.0f;
  const float c = g_radar_tw[L + i].x;  // cos is even: the table's real part
  return kind == 1 ? 0.5f - 0.5f * c : 0.54f - 0.46f * c;
}

// The same windows written as w(i) = a0 - a1 cos(2 pi i/L): (a0, a1).
__device__ __forceinline__ float2 window_coeffs(int kind) {
  if (kind == 0) return make_float2(1.0f, 0.0f);
  return kind == 1 ? make_float2(0.5f, 0.5f) : make_float2(0.54f, 0.46f);
}

}  // namespace radar
