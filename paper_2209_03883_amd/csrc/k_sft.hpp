// FPS-SFT, the sparse alternative to the periodogram (Sec. III-C).
//
// A slice of direction (alpha, beta) and offset (tau1, tau2) samples the LS
// estimate h[k, l] (subcarrier k, symbol l, ZC removed, Eq. 16) along
// t -> ((alpha t + tau1) mod N, (beta t + tau2) mod M), t < Q = lcm(N, M).  Its
// Q-point DFT is the projection of the 2-D spectrum X = DFT_N x DFT_M of h onto
// bins m = (alpha k1 Q/N + beta k2 Q/M) mod Q, each frequency weighted by
// Q/(NM) and by the offset phase exp(+2 pi i (k1 tau1/N + k2 tau2/M)).
//
// K5 (k5_sft_slices): gather, de-precode and divide the 3 * I slices of every
//    frame and run their Q-point DFTs.  These are linear in h, so all of them
//    run in parallel before any decoding.
// K6 (k6_sft_decode): one work-group per frame runs the recovery over the
//    directions in order: peel the known components off the three slices,
//    sort the bins by |S0|^2 (which also gives the median for the noise
//    threshold), test and decode the candidate bins in parallel, then merge
//    the accepted ones in bin order with one wavefront until k components
//    are known.
#pragma once

#include "device_common.hpp"
#include "fft.hpp"
#include "k_peaks.hpp"
#include "../../include/radar.h"

namespace radar {

constexpr int kSftMaxDirs = 16;
constexpr int kSftMaxK = 64;
constexpr int kSftDecodeThreads = 1024;

struct K5Args {
  const float2* Y;
  const float2* A;
  int64_t ld, frame_stride;
  float2* S;           // [F][I][3][Q]
  uint32_t* status;    // [F]
  int N, M, n_dirs, total;  // total = F * I * 3 slices
  uint32_t zc_root, zc_shift;
  int dir_a[kSftMaxDirs], dir_b[kSftMaxDirs];  // reduced to [0, N) and [0, M)
};

template <int Q>
struct K5Shape {
  static constexpr int T = Q / 16;                        // threads per slice
  static constexpr int BLOCK = T > 256 ? T : 256;
  static constexpr int TEAMS = BLOCK / T;
};

template <int Q>
__global__ void __launch_bounds__(K5Shape<Q>::BLOCK) k5_sft_slices(K5Args a) {
  using C = K5Shape<Q>;
  constexpr int T = C::T;
  __shared__ float2 lds_all[C::TEAMS * LdsSize<Q>::value];
  const int team = threadIdx.x / T;
  const int t = threadIdx.x - team * T;
  const int g = blockIdx.x * C::TEAMS + team;             // slice over all frames
  const bool active = g < a.total;
  const int gc = active ? g : 0;
  const int f = gc / (3 * a.n_dirs);
  const int rem = gc - f * 3 * a.n_dirs;
  const int dir = rem / 3;
  const int off = rem - dir * 3;                          // offsets (0,0), (1,0), (0,1)
  const int al = a.dir_a[dir], be = a.dir_b[dir];
  const int t1 = off == 1 ? 1 : 0, t2 = off == 2 ? 1 : 0;
  const float2* y = a.Y + (int64_t)f * a.frame_stride;
  const float2* x = a.A + (int64_t)f * a.frame_stride;
  float2* lds = lds_all + team * LdsSize<Q>::value;

  uint32_t st = 0;
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int tt = t + T * e;
    const int k = (al * tt + t1) & (a.N - 1);
    const int l = (be * tt + t2) & (a.M - 1);
    const int64_t idx = (int64_t)l * a.ld + k;
    const float2 yv = y[idx];
    const float2 av = x[idx];
    // conj(z_k) = W_{2N}^{m_k}, m_k = root*(k^2 + 2 q k) mod 2N (Eq. 23, even N);
    // root = 0 without precoding gives exactly 1
    const uint32_t uk = (uint32_t)k;
    const uint32_t m = (a.zc_root * (uk * uk + 2u * a.zc_shift * uk)) & (uint32_t)(2 * a.N - 1);
    const float2 hz = cmul(yv, twiddle(2 * a.N, (int)m));
    const float den = cabs2(av);
    st |= den == 0.0f ? 1u : 0u;
    const float inv = den == 0.0f ? 0.0f : __builtin_amdgcn_rcpf(den);
    v[e] = cscale(cmulc(hz, av), inv);                     // y conj(z) conj(a) / |a|^2
    st |= (__builtin_isfinite(v[e].x) && __builtin_isfinite(v[e].y)) ? 0u : 2u;
  }
  team_fft<Q, 16, false>(v, lds, t, active);
  if (!active) return;
  float2* out = a.S + (int64_t)g * Q;
#pragma unroll
  for (int e = 0; e < 16; ++e) out[t + T * e] = v[e];
  if (st && a.status) atomicOr(a.status + f, st);
}

struct K6Args {
  const float2* S;     // [F][I][3][Q]
  radar_peak* peaks;   // [F][k]
  int32_t* n_peaks;    // [F]
  int N, M, n_dirs, k;
  float thr_factor;    // -ln(pfa) / ln 2
  float tol;
  float floor_rel;     // numerically empty bins: power <= floor_rel * raw max
  int dir_a[kSftMaxDirs], dir_b[kSftMaxDirs];
};

__device__ __forceinline__ int sft_bin(int k1, int k2, int al, int be, int N, int M, int Q) {
  return (al * k1 * (Q / N) + be * k2 * (Q / M)) & (Q - 1);
}

// Descending bitonic sort of n (a power of two) keys in LDS by the whole block.
__device__ __forceinline__ void bitonic_sort_desc(uint64_t* key, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) {
        const int lo = 2 * i - (i & (stride - 1));       // first index of the pair
        const int hi = lo + stride;
        const bool desc = (lo & size) == 0;
        const uint64_t a = key[lo], b = key[hi];
        if ((a < b) == desc) {
          key[lo] = b;
          key[hi] = a;
        }
      }
    }
  }
  __syncthreads();
}

template <int Q>
__global__ void __launch_bounds__(kSftDecodeThreads) k6_sft_decode(K6Args a) {
  __shared__ float2 s_sl[3][Q];
  __shared__ uint64_t s_key[Q];
  __shared__ int32_t s_dec[Q];            // decoded k1 | k2 << 16 per sorted position, -1 = rejected
  __shared__ int s_fk1[kSftMaxK], s_fk2[kSftMaxK];
  __shared__ float2 s_fc[kSftMaxK];
  __shared__ int s_count;
  __shared__ float s_red[kSftDecodeThreads / 64];
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int N = a.N, M = a.M;
  const float scale = (float)Q / ((float)N * (float)M);   // a power of two: exact
  if (tid == 0) s_count = 0;

  for (int dir = 0; dir < a.n_dirs; ++dir) {
    __syncthreads();
    const int count0 = s_count;
    if (count0 >= a.k) break;
    const int al = a.dir_a[dir], be = a.dir_b[dir];
    const float2* src = a.S + ((int64_t)f * a.n_dirs + dir) * 3 * Q;
    float mx = 0.0f;
    for (int i = tid; i < 3 * Q; i += kSftDecodeThreads) {
      const float2 v = src[i];
      s_sl[i / Q][i % Q] = v;
      if (i < Q) mx = fmaxf(mx, cabs2(v));
    }
    const float floor_p = a.floor_rel * block_max_f32(mx, s_red);  // also orders the LDS writes
    // peel the known components, one offset per thread, in the order found
    if (tid < 3) {
      for (int j = 0; j < count0; ++j) {
        const int k1 = s_fk1[j], k2 = s_fk2[j];
        const int mb = sft_bin(k1, k2, al, be, N, M, Q);
        float2 ph = make_float2(1.0f, 0.0f);                  // exp(+2 pi i (k1 tau1/N + k2 tau2/M))
        if (tid == 1) ph = twiddle(N, (N - k1) & (N - 1));
        if (tid == 2) ph = twiddle(M, (M - k2) & (M - 1));
        s_sl[tid][mb] = csub(s_sl[tid][mb], cmul(cscale(s_fc[j], scale), ph));
      }
    }
    __syncthreads();
    for (int i = tid; i < Q; i += kSftDecodeThreads)
      s_key[i] = make_key(ord_bits(cabs2(s_sl[0][i])), (uint32_t)i);
    bitonic_sort_desc(s_key, Q);
    // median of the Q powers (mean of the two central values) and the threshold
    const float p_hi = ord_value((uint32_t)(s_key[Q / 2 - 1] >> 32));
    const float p_lo = ord_value((uint32_t)(s_key[Q / 2] >> 32));
    const float theta2 = a.thr_factor * (0.5f * (p_hi + p_lo));
    // test and decode every candidate position (a prefix of the sorted order)
    for (int j = tid; j < Q; j += kSftDecodeThreads) {
      const uint64_t key = s_key[j];
      const float p = ord_value((uint32_t)(key >> 32));
      const int mb = (int)(0xFFFFFFFFu - (uint32_t)key);
      int dec = -2;                                         // -2: below threshold (end of candidates)
      if (p >= theta2 && p > floor_p) {
        dec = -1;
        const float2 s0 = s_sl[0][mb], s1 = s_sl[1][mb], s2 = s_sl[2][mb];
        const float q0 = cabs2(s0);
        const float r1 = sqrtf(cabs2(s1) / q0), r2 = sqrtf(cabs2(s2) / q0);
        if (fabsf(r1 - 1.0f) <= a.tol && fabsf(r2 - 1.0f) <= a.tol) {
          const float2 c1 = cmulc(s1, s0), c2 = cmulc(s2, s0);  // arg(S1/S0), arg(S2/S0)
          constexpr float kInv2Pi = 0.15915494309189535f;
          const int k1 = (int)rintf((float)N * atan2f(c1.y, c1.x) * kInv2Pi) & (N - 1);
          const int k2 = (int)rintf((float)M * atan2f(c2.y, c2.x) * kInv2Pi) & (M - 1);
          if (sft_bin(k1, k2, al, be, N, M, Q) == mb) dec = k1 | (k2 << 16);
        }
      }
      s_dec[j] = dec;
    }
    __syncthreads();
    // merge in sorted order (one wavefront; lane q owns found slot q)
    if (tid < 64) {
      int count = count0;
      const float inv_scale = 1.0f / scale;
      bool stop = false;
      for (int j0 = 0; j0 < Q && !stop; j0 += 64) {
        const int j = j0 + tid;
        const int dec = j < Q ? s_dec[j] : -2;
        uint64_t endm = __ballot(dec == -2);
        uint64_t acc = __ballot(dec >= 0);
        const int lim = endm ? __builtin_ctzll(endm) : 64;  // candidates end here
        if (lim < 64) {
          acc &= (lim == 0) ? 0ull : (~0ull >> (64 - lim));
          stop = true;
        }
        while (acc) {
          const int b = __builtin_ctzll(acc);
          acc &= acc - 1;
          const int d = __shfl(dec, b);
          const int k1 = d & 0xFFFF, k2 = d >> 16;
          const int mb = (int)(0xFFFFFFFFu - (uint32_t)s_key[j0 + b]);
          const float2 c = cscale(s_sl[0][mb], inv_scale);
          const uint64_t same = __ballot(tid < count && s_fk1[tid] == k1 && s_fk2[tid] == k2);
          if (same) {
            const int q = __builtin_ctzll(same);
            if (tid == q) s_fc[q] = cadd(s_fc[q], c);
          } else {
            if (tid == count) {
              s_fk1[count] = k1;
              s_fk2[count] = k2;
              s_fc[count] = c;
            }
            ++count;
          }
          if (count >= a.k) {
            stop = true;
            break;
          }
        }
      }
      if (tid == 0) s_count = count;
    }
  }
  __syncthreads();
  // rank by (p descending, flat index ascending) and write the detections
  const int count = s_count;
  if (tid < count) {
    const int k1 = s_fk1[tid], k2 = s_fk2[tid];
    const float inv_nm = 1.0f / ((float)N * (float)M);
    const float p = cabs2(s_fc[tid]) * inv_nm;
    const int s = k2 < M / 2 ? k2 : k2 - M;
    const int r = (N - k1) & (N - 1);
    const uint32_t flat = (uint32_t)(s + M / 2) * (uint32_t)N + (uint32_t)r;
    const uint64_t key = make_key(ord_bits(p), flat);
    int rank = 0;
    for (int q = 0; q < count; ++q) {
      const int qk1 = s_fk1[q], qk2 = s_fk2[q];
      const float qp = cabs2(s_fc[q]) * inv_nm;
      const int qs = qk2 < M / 2 ? qk2 : qk2 - M;
      const int qr = (N - qk1) & (N - 1);
      const uint64_t qkey = make_key(ord_bits(qp), (uint32_t)(qs + M / 2) * (uint32_t)N + (uint32_t)qr);
      rank += qkey > key ? 1 : 0;
    }
    radar_peak pk;
    pk.s = s;
    pk.r = r;
    pk.p = p;
    pk.s_off = 0.0f;
    pk.r_off = 0.0f;
    a.peaks[(int64_t)f * a.k + rank] = pk;
  }
  if (tid == 0) a.n_peaks[f] = count;
}

}  // namespace radar
