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

// The device library's wavefront reduction (cross-lane moves within rows of
// 16 lanes, then across rows, the result read from one lane into scalar
// registers): no LDS round trips.  Every lane of the wavefront must be active.
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(unsigned long long);

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) { return __ockl_wfred_max_u64(v); }

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

// The k (<= 64) largest of n distinct keys key_at(j), j < n, by a 256-thread
// work-group: each wavefront ranks its share (j = 64 w + lane + 256 q) in k
// rounds of "largest key below the previous one" (no barriers), then
// wavefront 0 ranks the 4 k survivors the same way.  out[0..k) receives the
// keys in descending order, 0-padded; s_top holds 4 x 64 keys of scratch.
// Every thread must call it (two barriers); out is valid after it returns.
template <class KeyAt>
__device__ __forceinline__ void block_topk(int n, int k, const KeyAt& key_at, uint64_t (*s_top)[64],
                                           uint64_t* out) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint64_t last = ~0ull;
  int i = 0;
  for (; i < k; ++i) {
    uint64_t best = 0;
    for (int j = 64 * wave + lane; j < n; j += 256) {
      const uint64_t key = key_at(j);
      if (key < last && key > best) best = key;
    }
    best = wave_max_u64(best);
    if (lane == 0) s_top[wave][i] = best;
    if (best == 0) break;
    last = best;
  }
  for (int q = i + 1 + lane; q < k; q += 64) s_top[wave][q] = 0;
  __syncthreads();
  if (wave == 0) {
    last = ~0ull;
    for (i = 0; i < k; ++i) {
      uint64_t best = 0;
      for (int j = lane; j < 4 * k; j += 64) {
        const uint64_t key = s_top[j / k][j - (j / k) * k];
        if (key < last && key > best) best = key;
      }
      best = wave_max_u64(best);
      if (lane == 0) out[i] = best;
      last = best;
    }
  }
  __syncthreads();
}

// Nonzero candidate keys a frame's ranking gathers into LDS before it ranks
// them (beyond that it ranks the slots in global memory).
constexpr int kMergeCap = 4096;

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
                                                        int32_t* list, int32_t* cnt_out, float slack, int top_r) {
  extern __shared__ uint32_t s_dyn[];  // the row maxima, then the indices of profile peaks
  __shared__ uint64_t s_top[4][64];
  __shared__ uint64_t s_best[64];
  __shared__ int s_cnt[4];
  __shared__ int s_np;
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int mask = m_pad - 1;
  float* m = reinterpret_cast<float*>(s_dyn);
  uint32_t* pk = s_dyn + m_pad;
  if (tid == 0) s_np = 0;
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
  // the profile peaks (rows whose maximum is >= both neighbours'), gathered
  // in any order: the ranking below depends only on their keys
  for (int i = tid; i < m_pad; i += 256) {
    const float v = m[i];
    if (v >= m[(i - 1) & mask] && v >= m[(i + 1) & mask]) pk[atomicAdd(&s_np, 1)] = (uint32_t)i;
  }
  __syncthreads();
  const int np = s_np;
  block_topk(np, k, [&](int j) { const uint32_t i = pk[j]; return make_key(ord_bits(m[i]), i); }, s_top, s_best);
  const uint64_t kth = s_best[k - 1];
  float tau = kth ? ord_value((uint32_t)(kth >> 32)) : -__builtin_huge_valf();
  if (kth) tau -= fabsf(tau) * slack;

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
  if (top_r > 0 && total > top_r) {
    // a shortened first listing (peaks only, top_r <= 64): just the top_r
    // rows with the largest maxima, ascending; k_peak_second_listing adds
    // whatever else can hold a top-k peak
    __syncthreads();  // the ranking's reads of pk are done
    for (int i = lo; i < hi; ++i)
      if (m[i] >= tau) pk[pos++] = (uint32_t)i;
    __syncthreads();
    block_topk(total, top_r, [&](int j) { const uint32_t i = pk[j]; return make_key(ord_bits(m[i]), i); }, s_top,
               s_best);
    // rank by row index among the chosen (the keys are distinct)
    if (tid < top_r) {
      const uint32_t row = 0xFFFFFFFFu - (uint32_t)s_best[tid];
      int rank = 0;
      for (int q = 0; q < top_r; ++q) rank += (0xFFFFFFFFu - (uint32_t)s_best[q]) < row ? 1 : 0;
      out[rank] = (int32_t)row;
    }
    if (tid == 0) {
      cnt_out[f] = top_r;
      tau_out[f] = tau;
    }
    return;
  }
  for (int i = lo; i < hi; ++i)
    if (m[i] >= tau) out[pos++] = i;
  if (tid == 0) {
    cnt_out[f] = total;
    tau_out[f] = tau;
  }
}

// Peaks only: the second listing.  The first listing's rows [0, cnt[f]) have
// been recomputed and scanned, their k best candidates each in cand.  The
// k-th best of those, v, is a lower bound on the k-th peak (k distinct local
// maxima reach it), so a row can hold a top-k peak only if its recomputed
// maximum reaches v; the range stage's maximum m, which may fall short of it
// by the relative error `slack`, then reaches v / (1 + slack).  Every row
// that does and is not listed yet is appended, ascending; start[f] is set to
// the first of them and cnt[f] to the new end.  With fewer than k
// candidates found every remaining row is appended.  Grid F, 256 threads,
// dynamic LDS (m_pad + 31) / 32 words.
__global__ void __launch_bounds__(256) k_peak_second_listing(const float* rowmax, int m_pad, int k,
                                                             const uint64_t* cand, int32_t* list, int32_t* cnt,
                                                             int32_t* start, float slack) {
  extern __shared__ uint32_t s_bits[];  // the first listing's rows
  __shared__ uint64_t s_key[kMergeCap];
  __shared__ uint64_t s_top[4][64];
  __shared__ uint64_t s_best[64];
  __shared__ int s_cnt[4];
  __shared__ int s_n;
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int na = cnt[f];
  int32_t* lst = list + (int64_t)f * m_pad;
  const float* m = rowmax + (int64_t)f * m_pad;
  for (int j = tid; j < (m_pad + 31) / 32; j += 256) s_bits[j] = 0u;
  if (tid == 0) s_n = 0;
  __syncthreads();
  for (int j = tid; j < na; j += 256) atomicOr(&s_bits[lst[j] >> 5], 1u << (lst[j] & 31));
  const int count = na * k;
  const uint64_t* c = cand + (int64_t)f * m_pad * k;
  for (int j = tid; j < count; j += 256) {
    const uint64_t key = c[j];
    if (key) {
      const int p = atomicAdd(&s_n, 1);
      if (p < kMergeCap) s_key[p] = key;
    }
  }
  __syncthreads();
  const int n = s_n;
  if (n <= kMergeCap)
    block_topk(n, k, [&](int j) { return s_key[j]; }, s_top, s_best);
  else
    block_topk(count, k, [&](int j) { return c[j]; }, s_top, s_best);
  const uint64_t kth = s_best[k - 1];
  const float bound = kth ? ord_value((uint32_t)(kth >> 32)) / (1.0f + slack) : -__builtin_huge_valf();
  const int chunk = (m_pad + 255) / 256;
  const int lo = tid * chunk < m_pad ? tid * chunk : m_pad;
  const int hi = lo + chunk <= m_pad ? lo + chunk : m_pad;
  const auto open = [&](int i) { return m[i] >= bound && !((s_bits[i >> 5] >> (i & 31)) & 1u); };
  int cc = 0;
  for (int i = lo; i < hi; ++i) cc += open(i) ? 1 : 0;
  int incl = cc;
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
  int pos = na + before + incl - cc;
  for (int i = lo; i < hi; ++i)
    if (open(i)) lst[pos++] = i;
  if (tid == 0) {
    start[f] = na;
    cnt[f] = na + total;
  }
}

// Columns c0-1 .. c0+8 of a row (cyclic; c0 a multiple of 8, n_pad >= 8 a
// power of two): from global memory as two 16-byte loads and two single
// values, from LDS value by value.
__device__ __forceinline__ void load_cols10(const RADAR_GLOBAL float* row, int c0, int n_pad, float (&a)[10]) {
  const radar_v4 x = *(const RADAR_GLOBAL radar_v4*)(row + c0);
  const radar_v4 y = *(const RADAR_GLOBAL radar_v4*)(row + c0 + 4);
  a[0] = row[(c0 - 1) & (n_pad - 1)];
  a[9] = row[(c0 + 8) & (n_pad - 1)];
  a[1] = x.x, a[2] = x.y, a[3] = x.z, a[4] = x.w;
  a[5] = y.x, a[6] = y.y, a[7] = y.z, a[8] = y.w;
}
__device__ __forceinline__ void load_cols10(const float* row, int c0, int n_pad, float (&a)[10]) {
  a[0] = row[(c0 - 1) & (n_pad - 1)];
  a[9] = row[(c0 + 8) & (n_pad - 1)];
#pragma unroll
  for (int u = 0; u < 8; ++u) a[u + 1] = row[c0 + u];
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
  // eight contiguous columns per thread at a time: the three rows' values
  // at columns c0-1 .. c0+8 are loaded once (two 16-byte loads and two
  // single values per row, every load issued before any test), and each
  // cell's 3 x 3 neighbourhood is read from them
  int mine = 0;
  for (int c0 = 8 * (int)threadIdx.x; c0 < n_pad; c0 += 8 * (int)blockDim.x) {
    float a[3][10];
    load_cols10(rm, c0, n_pad, a[0]);
    load_cols10(r0, c0, n_pad, a[1]);
    load_cols10(rp, c0, n_pad, a[2]);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float v = a[1][u + 1];
      bool pk = v >= th;
#pragma unroll
      for (int q = 0; q < 3; ++q) pk = pk && v >= a[0][u + q] && v >= a[2][u + q];
      pk = pk && v >= a[1][u] && v >= a[1][u + 2];
      s_ord[c0 + u] = pk ? ord_bits(v) : 0u;
      mine += pk ? 1 : 0;
    }
  }
  // how many candidates does the row hold?
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
    for (int c0 = 8 * (int)threadIdx.x; c0 < n_pad; c0 += 8 * (int)blockDim.x)
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (s_ord[c0 + u]) out[pos++] = make_key(s_ord[c0 + u], flat0 + (uint32_t)(c0 + u));
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
  // a contiguous run of the (ascending) list per work-group: listed rows
  // come in runs of neighbours, so the rows above and below one listed row
  // are the listed rows next to it, read moments before by the same
  // work-group (cache hits rather than HBM reads)
  const int per = (count + (int)gridDim.x - 1) / (int)gridDim.x;
  const int j0 = (int)blockIdx.x * per;
  const int j1 = j0 + per < count ? j0 + per : count;
  for (int j = j0; j < j1; ++j) {
    const int row = list[(int64_t)f * m_pad + j];
    const RADAR_GLOBAL float* rm = base + (int64_t)((row - 1) & (m_pad - 1)) * n_pad;
    const RADAR_GLOBAL float* r0 = base + (int64_t)row * n_pad;
    const RADAR_GLOBAL float* rp = base + (int64_t)((row + 1) & (m_pad - 1)) * n_pad;
    row_candidates(rm, r0, rp, n_pad, k, th, (uint32_t)row * (uint32_t)n_pad, s_ord, red, s_cnt,
                   cand + ((int64_t)f * m_pad + j) * k);
  }
}

// Step 4: the k best keys over the scanned rows of a frame (grid F, 256
// threads).  The scanned rows leave k slots each, mostly 0-padding: the
// nonzero keys are first gathered into LDS (up to kMergeCap of them; beyond
// that the ranking reads the slots in global memory) and ranked there.  With
// inv_sum (threshold detection, Eq. 18) the list stops at the first peak
// below eta = eta_factor * sum_l inv_sum[f][l]; the peaks come in descending
// P, so what is kept is exactly the top-k local maxima at or above eta.
__global__ void __launch_bounds__(256) k_peak_merge(const uint64_t* cand, const int32_t* cnt, int m_pad, int n_pad,
                                                    int k, radar_peak* peaks, int32_t* n_peaks,
                                                    const FrameRef* refs, const float* inv_sum, int M,
                                                    float eta_factor) {
  __shared__ uint64_t s_key[kMergeCap];
  __shared__ uint64_t s_top[4][64];
  __shared__ uint64_t s_best[64];
  __shared__ int s_n;
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int count = cnt[f] * k;
  const uint64_t* c = cand + (int64_t)f * m_pad * k;
  if (tid == 0) s_n = 0;
  __syncthreads();
  for (int j = tid; j < count; j += 256) {
    const uint64_t key = c[j];
    if (key) {
      const int pos = atomicAdd(&s_n, 1);
      if (pos < kMergeCap) s_key[pos] = key;
    }
  }
  __syncthreads();
  const int n = s_n;
  if (n <= kMergeCap)
    block_topk(n, k, [&](int j) { return s_key[j]; }, s_top, s_best);
  else
    block_topk(count, k, [&](int j) { return c[j]; }, s_top, s_best);
  if (tid >= 64) return;
  float eta = -__builtin_huge_valf();
  if (inv_sum) {
    float acc = 0.0f;  // fixed order: lane-strided partial sums, then a butterfly
    for (int l = tid; l < M; l += 64) acc += inv_sum[(int64_t)f * M + l];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
    eta = (refs ? refs[f].eta_factor : eta_factor) * acc;
  }
  // lane i emits the i-th best; the kept peaks are a prefix (keys and values
  // both descend)
  const uint64_t best = tid < k ? s_best[tid] : 0;
  const float p = ord_value((uint32_t)(best >> 32));
  const bool keep = best != 0 && !(p < eta);
  const uint64_t kept = __ballot(keep);
  const int n_kept = (int)__builtin_popcountll(kept);
  if (tid < n_kept) {
    const uint32_t flat = 0xFFFFFFFFu - (uint32_t)best;
    radar_peak pk;
    pk.s = (int32_t)(flat / (uint32_t)n_pad) - (m_pad >> 1);
    pk.r = (int32_t)(flat % (uint32_t)n_pad);
    pk.p = p;
    pk.s_off = 0.0f;
    pk.r_off = 0.0f;
    (refs ? refs[f].peaks : peaks + (int64_t)f * k)[tid] = pk;
  }
  if (tid == 0) *(refs ? refs[f].n_peaks : n_peaks + f) = n_kept;
}

}  // namespace radar
