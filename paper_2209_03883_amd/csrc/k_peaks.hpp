// Peak extraction: the k largest 3x3 cyclic local maxima of a periodogram,
// ranked by (value descending, flat index ascending).
//
// A candidate is encoded as a 64-bit key whose high word is an order-preserving
// image of the float value and whose low word is 0xFFFFFFFF - flat index, so
// "larger key" is exactly "ranks first".  Key 0 means "no candidate".
//
//   k_peak_rows   one work-group per row: marks the row's local maxima (its
//                 two neighbour rows are read too) and emits the row's k best
//                 keys.  The k best peaks of a frame are among the union of the
//                 rows' k best, so this is exact.
//   k_peak_merge  one work-group per frame: the k best keys over all rows.
#pragma once

#include "device_common.hpp"
#include "../../include/radar.h"

namespace radar {

// Order-preserving float -> uint32 (the result is never 0: that value is
// reserved for "no candidate").
__device__ __forceinline__ uint32_t ord_bits(float v) {
  if (v == 0.0f) v = 0.0f;  // -0 ranks like +0
  const uint32_t u = __float_as_uint(v);
  const uint32_t o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return o ? o : 1u;
}
__device__ __forceinline__ float ord_value(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

__device__ __forceinline__ uint64_t make_key(uint32_t ord, uint32_t flat) {
  return ((uint64_t)ord << 32) | (uint64_t)(0xFFFFFFFFu - flat);
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    v = o > v ? o : v;
  }
  return v;
}

// Work-group maximum; every thread gets the result.  `red` holds one slot per wave.
__device__ __forceinline__ uint64_t block_max_u64(uint64_t v, uint64_t* red) {
  v = wave_max_u64(v);
  const int wave = threadIdx.x >> 6;
  const int nwaves = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  uint64_t r = red[0];
  for (int i = 1; i < nwaves; ++i) r = red[i] > r ? red[i] : r;
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(256) k_peak_rows(const float* P, int64_t p_stride, int m_pad, int n_pad,
                                                   int k, uint64_t* cand) {
  extern __shared__ uint32_t s_ord[];  // n_pad entries, 0 = not a local maximum
  __shared__ uint64_t red[4];
  const int f = blockIdx.y;
  const int row = blockIdx.x;
  const float* base = P + (int64_t)f * p_stride;
  const float* rm = base + (int64_t)((row - 1) & (m_pad - 1)) * n_pad;
  const float* r0 = base + (int64_t)row * n_pad;
  const float* rp = base + (int64_t)((row + 1) & (m_pad - 1)) * n_pad;
  for (int r = threadIdx.x; r < n_pad; r += blockDim.x) {
    const int rl = (r - 1) & (n_pad - 1);
    const int rr = (r + 1) & (n_pad - 1);
    const float v = r0[r];
    const bool pk = v >= r0[rl] && v >= r0[rr] && v >= rm[rl] && v >= rm[r] && v >= rm[rr] &&
                    v >= rp[rl] && v >= rp[r] && v >= rp[rr];
    s_ord[r] = pk ? ord_bits(v) : 0u;
  }
  __syncthreads();
  uint64_t* out = cand + ((int64_t)f * m_pad + row) * k;
  const uint32_t flat0 = (uint32_t)row * (uint32_t)n_pad;
  uint64_t last = ~0ull;
  int i = 0;
  for (; i < k; ++i) {
    uint64_t best = 0;
    for (int r = threadIdx.x; r < n_pad; r += blockDim.x) {
      const uint32_t o = s_ord[r];
      if (o) {
        const uint64_t key = make_key(o, flat0 + (uint32_t)r);
        if (key < last && key > best) best = key;
      }
    }
    best = block_max_u64(best, red);
    if (threadIdx.x == 0) out[i] = best;
    if (best == 0) break;
    last = best;
  }
  if (threadIdx.x == 0)
    for (int j = i + 1; j < k; ++j) out[j] = 0;
}

__global__ void __launch_bounds__(1024) k_peak_merge(const uint64_t* cand, int m_pad, int n_pad, int k,
                                                     radar_peak* peaks, int32_t* n_peaks) {
  __shared__ uint64_t red[16];
  const int f = blockIdx.x;
  const int count = m_pad * k;
  const uint64_t* c = cand + (int64_t)f * count;
  uint64_t last = ~0ull;
  int i = 0;
  for (; i < k; ++i) {
    uint64_t best = 0;
    for (int j = threadIdx.x; j < count; j += blockDim.x) {
      const uint64_t key = c[j];
      if (key < last && key > best) best = key;
    }
    best = block_max_u64(best, red);
    if (best == 0) break;
    if (threadIdx.x == 0) {
      const uint32_t flat = 0xFFFFFFFFu - (uint32_t)best;
      radar_peak pk;
      pk.s = (int32_t)(flat / (uint32_t)n_pad) - (m_pad >> 1);
      pk.r = (int32_t)(flat % (uint32_t)n_pad);
      pk.p = ord_value((uint32_t)(best >> 32));
      pk.s_off = 0.0f;
      pk.r_off = 0.0f;
      peaks[(int64_t)f * k + i] = pk;
    }
    last = best;
  }
  if (threadIdx.x == 0) n_peaks[f] = i;
}

}  // namespace radar
