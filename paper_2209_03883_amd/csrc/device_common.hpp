// Device-side helpers shared by every radar kernel: complex arithmetic on
// float2 and the library's twiddle table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// The twiddle table holds W^t = exp(-2*pi*i*t / RADAR_TW_LMAX) for
// t in [0, RADAR_TW_LMAX), each value computed on the host in double
// precision and rounded once to float.  W_L^x for a power-of-two L that
// divides RADAR_TW_LMAX is entry x * (RADAR_TW_LMAX / L).
#define RADAR_TW_LOG2 14
#define RADAR_TW_LMAX (1 << RADAR_TW_LOG2)

extern __device__ float2 g_radar_tw[RADAR_TW_LMAX];

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

// exp(-2*pi*i*t/L) for L = RADAR_TW_LMAX >> shift, t < L.
__device__ __forceinline__ float2 twiddle(int t, int shift) { return g_radar_tw[t << shift]; }

// Periodic window value w(i) of length L = RADAR_TW_LMAX >> shift
// (Hann: 0.5 - 0.5 cos(2 pi i/L); Hamming: 0.54 - 0.46 cos(2 pi i/L); rect: 1).
__device__ __forceinline__ float window_value(int kind, int i, int shift) {
  if (kind == 0) return 1.0f;
  const float c = g_radar_tw[i << shift].x;  // cos is even: the table's real part
  return kind == 1 ? 0.5f - 0.5f * c : 0.54f - 0.46f * c;
}

}  // namespace radar
