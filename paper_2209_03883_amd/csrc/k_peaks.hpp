// Peak extraction: the k largest 3x3 cyclic local maxima of a periodogram,
// ranked by (value descending, flat index ascending).
//
// A candidate is encoded as a 64-bit key whose high word is an order-preserving
// image of the float value and whose low word is 0xFFFFFFFF - flat index, so
// "larger key" is exactly "ranks first".  Key 0 means "no candidate".
//
// Exact search without scanning every row:
//   1. m_s = max of row s (written by the range kernel, or k_row_max).
//   2. If m_s >= m_{s-1} and m_s >= m_{s+1} (cyclically), the cell holding m_s
//      is >= all its 8 neighbours, i.e. a local maximum of P.  Distinct such
//      rows give distinct local maxima, so the k-th largest of these m_s is a
//      lower bound tau on the k-th largest local maximum (tau = -inf when
//      fewer than k rows qualify).
//   3. Every local maximum >= tau lies in a row with m_s >= tau: only those
//      rows are scanned, each for its k best local maxima >= tau.
//   4. The k best over the scanned rows are the answer.
// (k_peak_threshold does 2, k_peak_rows_listed 3, k_peak_merge 4.)
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

__device__ __forceinline__ float block_max_f32(float v, float* red) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v = fmaxf(v, __shfl_xor(v, m));
  const int nwaves = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = red[0];
  for (int i = 1; i < nwaves; ++i) r = fmaxf(r, red[i]);
  __syncthreads();
  return r;
}

// Row maxima of arbitrary periodograms (used when the range kernel did not
// produce them).  Grid (m_pad, F), 256 threads.
__global__ void __launch_bounds__(256) k_row_max(const float* P, int64_t p_stride, int m_pad, int n_pad,
                                                 float* rowmax, const FrameRef* refs) {
  __shared__ float red[4];
  const int f = blockIdx.y, row = blockIdx.x;
  const RADAR_GLOBAL float* r0 = gptr(refs ? refs[f].P : P + (int64_t)f * p_stride) + (int64_t)row * n_pad;
  float mx = -__builtin_huge_valf();
  for (int r = threadIdx.x; r < n_pad; r += blockDim.x) mx = fmaxf(mx, r0[r]);
  mx = block_max_f32(mx, red);
  if (threadIdx.x == 0) rowmax[(int64_t)f * m_pad + row] = mx;
}

// Step 2 and the row list of step 3 (grid F, 256 threads, dynamic LDS 2 m_pad
// words).  The row maxima are copied into LDS first, eight loads per thread
// in flight at a time; profile peaks are marked in LDS with strided row
// ownership; the k-th largest comes from k rounds of work-group maxima; the
// row list is written in ascending order from contiguous row chunks.
//
// slack > 0 (peaks only, P not materialised): the row maxima come from the
// range kernel while the scan reads rows recomputed by another kernel, which
// may differ by a few FP32 ulps.  The bound is then lowered to
// tau (1 - slack), for the listing and for the scan alike, so that a local
// maximum sitting at tau whose recomputed value lands just below it is still
// found; the merge keeps only the k best, so the extra candidates cost only
// scanning.
__global__ void __launch_bounds__(256) k_peak_threshold(const float* rowmax, int m_pad, int k, float* tau_out,
                                                        int32_t* list, int32_t* cnt_out, float slack) {
  extern __shared__ uint32_t s_prof[];  // ord bits of profile peaks, 0 elsewhere; then the row maxima
  __shared__ uint64_t red[4];
  __shared__ int s_cnt[4];
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int mask = m_pad - 1;
  float* m = reinterpret_cast<float*>(s_prof + m_pad);
  {
    const float* g = rowmax + (int64_t)f * m_pad;
    for (int base = tid; base < m_pad; base += 8 * 256) {
      float tv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) tv[u] = g[base + u * 256 < m_pad ? base + u * 256 : 0];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (base + u * 256 < m_pad) m[base + u * 256] = tv[u];
    }
  }
  __syncthreads();
  for (int i = tid; i < m_pad; i += 256) {
    const float v = m[i];
    s_prof[i] = (v >= m[(i - 1) & mask] && v >= m[(i + 1) & mask]) ? ord_bits(v) : 0u;
  }
  __syncthreads();
  uint64_t last = ~0ull;
  int found = 0;
  for (; found < k; ++found) {
    uint64_t best = 0;
    for (int i = tid; i < m_pad; i += 256) {
      const uint32_t o = s_prof[i];
      if (o) {
        const uint64_t key = make_key(o, (uint32_t)i);
        if (key < last && key > best) best = key;
      }
    }
    best = block_max_u64(best, red);
    if (best == 0) break;
    last = best;
  }
  float tau = found == k ? ord_value((uint32_t)(last >> 32)) : -__builtin_huge_valf();
  if (found == k) tau -= fabsf(tau) * slack;

  const int chunk = (m_pad + 255) / 256;
  const int lo = tid * chunk < m_pad ? tid * chunk : m_pad;
  const int hi = lo + chunk <= m_pad ? lo + chunk : m_pad;
  int c = 0;
  for (int i = lo; i < hi; ++i) c += m[i] >= tau ? 1 : 0;
  int incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int up = __shfl_up(incl, off);
    if ((tid & 63) >= off) incl += up;
  }
  if ((tid & 63) == 63) s_cnt[tid >> 6] = incl;
  __syncthreads();
  int before = 0, total = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < (tid >> 6)) before += s_cnt[w];
    total += s_cnt[w];
  }
  int pos = before + incl - c;
  int32_t* out = list + (int64_t)f * m_pad;
  for (int i = lo; i < hi; ++i)
    if (m[i] >= tau) out[pos++] = i;
  if (tid == 0) {
    cnt_out[f] = total;
    tau_out[f] = tau;
  }
}

// Step 3 for one listed row: its exact local maxima >= th among the rows
// above (rm), at (r0) and below (rp), k best of them to out[0..k) (key 0
// pads).  Called by every thread of the work-group (256 threads; it contains
// barriers); s_ord holds n_pad words of scratch.  Row pointers may be global
// or LDS.
template <class RowPtr>
__device__ __forceinline__ void row_candidates(RowPtr rm, RowPtr r0, RowPtr rp, int n_pad, int k, float th,
                                               uint32_t flat0, uint32_t* s_ord, uint64_t* red, int* s_cnt,
                                               uint64_t* out) {
  // eight columns per thread at a time, all nine values of each 3 x 3
  // neighbourhood loaded before any test (unconditional loads, columns
  // clamped in bounds; the rows are L2-resident), so the loads overlap
  // instead of waiting one by one
  for (int base = threadIdx.x; base < n_pad; base += 8 * (int)blockDim.x) {
    float nb[8][9];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int r = base + u * (int)blockDim.x;
      const int rc = r < n_pad ? r : 0;
      const int rl = (rc - 1) & (n_pad - 1);
      const int rr = (rc + 1) & (n_pad - 1);
      nb[u][0] = r0[rc];
      nb[u][1] = r0[rl];
      nb[u][2] = r0[rr];
      nb[u][3] = rm[rl];
      nb[u][4] = rm[rc];
      nb[u][5] = rm[rr];
      nb[u][6] = rp[rl];
      nb[u][7] = rp[rc];
      nb[u][8] = rp[rr];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int r = base + u * (int)blockDim.x;
      if (r < n_pad) {
        const float v = nb[u][0];
        bool pk = v >= th;
#pragma unroll
        for (int q = 1; q < 9; ++q) pk = pk && v >= nb[u][q];
        s_ord[r] = pk ? ord_bits(v) : 0u;
      }
    }
  }
  // how many candidates does the row hold?
  int mine = 0;
  for (int r = threadIdx.x; r < n_pad; r += blockDim.x) mine += s_ord[r] ? 1 : 0;
  __syncthreads();
  int incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int up = __shfl_up(incl, off);
    if ((threadIdx.x & 63) >= off) incl += up;
  }
  if ((threadIdx.x & 63) == 63) s_cnt[threadIdx.x >> 6] = incl;
  __syncthreads();
  int total = 0, before = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < (int)(threadIdx.x >> 6)) before += s_cnt[w];
    total += s_cnt[w];
  }
  int i = 0;
  if (total <= k) {
    // few candidates: write them all (the merge ranks them), pad with 0
    int pos = before + incl - mine;
    for (int r = threadIdx.x; r < n_pad; r += blockDim.x)
      if (s_ord[r]) out[pos++] = make_key(s_ord[r], flat0 + (uint32_t)r);
    for (int q = total + (int)threadIdx.x; q < k; q += blockDim.x) out[q] = 0;
    i = k;  // nothing left to pad below
  } else {
    uint64_t last = ~0ull;
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
  }
  if (threadIdx.x == 0)
    for (int q = i + 1; q < k; ++q) out[q] = 0;
  __syncthreads();  // s_ord is rewritten for the next row
}

// Step 3: exact local maxima >= tau of the listed rows, k best per row.
// Grid (G, F), 256 threads, dynamic LDS n_pad words.  Output
// cand[f][j][0..k) for list entry j (key 0 pads).
__global__ void __launch_bounds__(256) k_peak_rows_listed(const float* P, int64_t p_stride, int m_pad, int n_pad,
                                                          int k, const float* tau, const int32_t* list,
                                                          const int32_t* cnt, uint64_t* cand,
                                                          const FrameRef* refs) {
  extern __shared__ uint32_t s_ord[];  // n_pad entries, 0 = not a candidate
  __shared__ uint64_t red[4];
  __shared__ int s_cnt[4];
  const int f = blockIdx.y;
  const int count = cnt[f];
  const float th = tau[f];
  const RADAR_GLOBAL float* base = gptr(refs ? refs[f].P : P + (int64_t)f * p_stride);
  for (int j = blockIdx.x; j < count; j += gridDim.x) {
    const int row = list[(int64_t)f * m_pad + j];
    const RADAR_GLOBAL float* rm = base + (int64_t)((row - 1) & (m_pad - 1)) * n_pad;
    const RADAR_GLOBAL float* r0 = base + (int64_t)row * n_pad;
    const RADAR_GLOBAL float* rp = base + (int64_t)((row + 1) & (m_pad - 1)) * n_pad;
    row_candidates(rm, r0, rp, n_pad, k, th, (uint32_t)row * (uint32_t)n_pad, s_ord, red, s_cnt,
                   cand + ((int64_t)f * m_pad + j) * k);
  }
}

// Step 4: the k best keys over the scanned rows of a frame, one wavefront per
// frame (grid F, 64 threads).  With inv_sum (threshold detection, Eq. 18) the
// list stops at the first peak below eta = eta_factor * sum_l inv_sum[f][l];
// the peaks come in descending P, so what is kept is exactly the top-k local
// maxima at or above eta.
__global__ void __launch_bounds__(64) k_peak_merge(const uint64_t* cand, const int32_t* cnt, int m_pad, int n_pad,
                                                   int k, radar_peak* peaks, int32_t* n_peaks,
                                                   const FrameRef* refs, const float* inv_sum, int M,
                                                   float eta_factor) {
  const int f = blockIdx.x;
  const int count = cnt[f] * k;
  const uint64_t* c = cand + (int64_t)f * m_pad * k;
  float eta = -__builtin_huge_valf();
  if (inv_sum) {
    float acc = 0.0f;  // fixed order: lane-strided partial sums, then a butterfly
    for (int l = threadIdx.x; l < M; l += 64) acc += inv_sum[(int64_t)f * M + l];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
    eta = (refs ? refs[f].eta_factor : eta_factor) * acc;
  }
  uint64_t last = ~0ull;
  int i = 0;
  for (; i < k; ++i) {
    uint64_t best = 0;
    for (int j = threadIdx.x; j < count; j += 64) {
      const uint64_t key = c[j];
      if (key < last && key > best) best = key;
    }
    best = wave_max_u64(best);
    if (best == 0) break;
    const float p = ord_value((uint32_t)(best >> 32));
    if (p < eta) break;
    if (threadIdx.x == 0) {
      const uint32_t flat = 0xFFFFFFFFu - (uint32_t)best;
      radar_peak pk;
      pk.s = (int32_t)(flat / (uint32_t)n_pad) - (m_pad >> 1);
      pk.r = (int32_t)(flat % (uint32_t)n_pad);
      pk.p = p;
      pk.s_off = 0.0f;
      pk.r_off = 0.0f;
      (refs ? refs[f].peaks : peaks + (int64_t)f * k)[i] = pk;
    }
    last = best;
  }
  if (threadIdx.x == 0) *(refs ? refs[f].n_peaks : n_peaks + f) = i;
}

}  // namespace radar
