// Device-side helpers shared by every radar kernel: complex arithmetic on
// float2 and the library's twiddle table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/radar.h"

// The twiddle table.  Every value is computed on the host in double precision
// and rounded once to float.  Three sections, laid out so that the entries a
// wavefront reads in one instruction are contiguous across its lanes:
//
//  power   g[L + x] = W_L^x = exp(-2 pi i x/L),  L = 1, 2, 4, ..., LMAX, x < L.
//  stage   for a Stockham stage of radix R = 2^r after span NS = 2^a:
//          g[stage_offset(a, r) + m*NS + k] = W_{NS*R}^{k*m},  m < R, k < NS.
//  phase   for a padding factor F = 2^p and length N = 2^n:
//          g[phase_offset(n, p) + b*N + k] = W_{F*N}^{k*b},  b < F, k < N.
#define RADAR_TW_LOG2 14
#define RADAR_TW_LMAX (1 << RADAR_TW_LOG2)

namespace radar {

constexpr int kTwPowerEntries = 2 * RADAR_TW_LMAX;

constexpr int stage_block(int a, int r) { return (1 << (a + r)) <= RADAR_TW_LMAX ? (1 << (a + r)) : 0; }
constexpr int stage_offset(int a, int r) {
  int off = kTwPowerEntries;
  for (int i = 0; i < a; ++i)
    for (int j = 1; j <= 4; ++j) off += stage_block(i, j);
  for (int j = 1; j < r; ++j) off += stage_block(a, j);
  return off;
}
constexpr int kTwStageEnd = stage_offset(RADAR_TW_LOG2, 1);

// phase blocks for n = 4..12 (N = 16..4096) and p = 1..3 (F = 2, 4, 8)
constexpr int phase_offset(int n, int p) {
  int off = kTwStageEnd;
  for (int i = 4; i < n; ++i)
    for (int j = 1; j <= 3; ++j) off += (1 << (i + j));
  for (int j = 1; j < p; ++j) off += (1 << (n + j));
  return off;
}
constexpr int kTwEntries = phase_offset(13, 1);

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

}  // namespace radar

#define RADAR_TW_ENTRIES (radar::kTwEntries)

extern __device__ float2 g_radar_tw[RADAR_TW_ENTRIES];

namespace radar {

// Per-frame buffers of one job of a batch with uneven shapes (device memory).
// Kernels given a table of these address frame f through refs[f] instead of
// base + f * stride.
struct FrameRef {
  const float2* Y;
  const float2* A;
  float* P;
  radar_peak* peaks;
  int32_t* n_peaks;
  uint32_t* status;
  float eta_factor;  // threshold detection: eta = eta_factor * sum of the frame's 1/|a|^2
};

// Pointers read from a FrameRef table are generic to the compiler.  The hot
// loads and stores go through pointers typed in the global address space, so
// they stay global (not flat) accesses, whose completion the LDS waits do not
// track.
#define RADAR_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ RADAR_GLOBAL T* gptr(T* p) {
  return (RADAR_GLOBAL T*)p;
}
typedef float radar_v2 __attribute__((ext_vector_type(2)));
typedef float radar_v4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float2 gload2(const RADAR_GLOBAL float2* p) {
  const radar_v2 v = *(const RADAR_GLOBAL radar_v2*)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gstore2(RADAR_GLOBAL float* p, float a, float b) {
  *(RADAR_GLOBAL radar_v2*)p = radar_v2{a, b};
}
__device__ __forceinline__ void gstore4(RADAR_GLOBAL float* p, float a, float b, float c, float d) {
  *(RADAR_GLOBAL radar_v4*)p = radar_v4{a, b, c, d};
}
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
__device__ __forceinline__ float2 twiddle(int L, int x) { return g_radar_tw[(unsigned)(L + x)]; }

// W_{NS*R}^{k*m} from the stage section.
template <int NS, int R>
__device__ __forceinline__ float2 stage_twiddle(int k, int m) {
  constexpr int off = stage_offset(ilog2c(NS), ilog2c(R));
  return g_radar_tw[(unsigned)(off + m * NS + k)];
}

// W_{F*N}^{k*b} from the phase section.
template <int N, int F>
__device__ __forceinline__ float2 phase_twiddle(int b, int k) {
  constexpr int off = phase_offset(ilog2c(N), ilog2c(F));
  return g_radar_tw[(unsigned)(off + b * N + k)];
}

// W_L^m for 0 <= m < L as the product of two small-table entries
// W_L^{m - m mod 64} * W_L^{m mod 64} (keeps a scattered lookup inside a few cache lines).
__device__ __forceinline__ float2 twiddle_split(int L, int m) {
  if (L <= 64) return twiddle(L, m);
  return cmul(twiddle(L >> 6, m >> 6), twiddle(L, m & 63));
}

// Periodic window value w(i) of length L (a power of two):
// Hann 0.5 - 0.5 cos(2 pi i/L); Hamming 0.54 - 0.46 cos(2 pi i/L); rect 1.
__device__ __forceinline__ float window_value(int kind, int i, int L) {
  if (kind == 0) return 1.0f;
  const float c = g_radar_tw[(unsigned)(L + i)].x;  // cos is even: the table's real part
  return kind == 1 ? 0.5f - 0.5f * c : 0.54f - 0.46f * c;
}

// The same windows written as w(i) = a0 - a1 cos(2 pi i/L): (a0, a1).
__device__ __forceinline__ float2 window_coeffs(int kind) {
  if (kind == 0) return make_float2(1.0f, 0.0f);
  return kind == 1 ? make_float2(0.5f, 0.5f) : make_float2(0.54f, 0.46f);
}

}  // namespace radar
