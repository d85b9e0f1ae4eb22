// FPS-SFT for any frame size (Sec. III-C: slices of length Q = lcm(N, M)),
// e.g. Table I's N = 2048 subcarriers by M = 560 symbols, Q = 71,680.
//
// The Q-point DFT of a slice.  Q = P R with P the largest power of two
// dividing Q and R odd, so gcd(P, R) = 1 and the prime-factor (Good-Thomas)
// mapping splits the DFT into a P-point and an R-point DFT with no twiddles
// between them:
//   input   t = (n1 R + n2 P) mod Q,                 n1 < P, n2 < R
//   output  m = (k1 R (R^-1 mod P) + k2 P (P^-1 mod R)) mod Q
//   S[m]  = sum_{n2} W_R^{n2 k2} sum_{n1} W_P^{n1 k1} s[t]
// (the products of the exponent reduce mod Q to R n1 k1 and P n2 k2 because
// R (R^-1 mod P) = 1 mod P and P (P^-1 mod R) = 1 mod R).  Pass 1 runs the
// P-point transforms with the library's team FFT, pass 2 the R-point DFTs
// directly (R is small).
//
// The recovery (k6g_sft_decode) is the same sequence of decisions as the
// power-of-two decoder, with the slices left in global memory: the known
// components are peeled through a per-bin correction table (a bitmap marks
// the bins), the median of |S0|^2 comes from a radix selection, and the bins
// above the threshold are gathered, sorted and merged in rounds of at most
// kSftGCap in descending order.
#pragma once

#include "k_sft.hpp"

namespace radar {

constexpr int kSftGMaxQ = 1 << 17;   // slice length of the general path
constexpr int kSftGMaxR = 255;       // largest odd factor R of Q
constexpr int kSftGCap = 4096;       // candidate bins sorted per round

struct K5gArgs {
  const float2* Y;
  const float2* A;
  int64_t ld, frame_stride;
  const float2* zc;    // conj(z_k), k < N, or null (no precoding)
  const float2* wr;    // W_R^x, x < R
  float2* Z;           // [slice][P][R] after pass 1
  float2* S;           // [slice][Q] spectra
  uint32_t* status;    // [F]
  int N, M, Q, P, R, n_dirs, total;  // total = F * n_dirs * 3 slices
  int r_inv, p_inv;    // R^-1 mod P, P^-1 mod R
  int dir_a[kSftMaxDirs], dir_b[kSftMaxDirs];
};

// conj(z_k) of Eq. 23 for any N, from the exact integer phase index
// m_k = r (k^2 + 2qk) mod 2N (N even) or r (k(k+1) + 2qk) mod 2N (N odd),
// z_k = exp(i pi m_k / N), in FP64 rounded once; and W_R^x = exp(-2 pi i x/R).
// root and shift reduced to [0, 2N) by the host; root 0 = no precoding.
__global__ void k_sft_tables(int N, int64_t root, int64_t shift, int R, float2* zc, float2* wr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (zc && i < N) {
    const int64_t k = i, two_n = 2 * (int64_t)N;
    const int64_t base = (N % 2 == 0) ? k * k : k * (k + 1);
    const int64_t m = (root * ((base + 2 * shift * k) % two_n)) % two_n;
    double s, c;
    sincospi((double)m / (double)N, &s, &c);
    zc[i] = make_float2((float)c, (float)-s);
  }
  if (i < R) {
    double s, c;
    sincospi(2.0 * (double)i / (double)R, &s, &c);
    wr[i] = make_float2((float)c, (float)-s);
  }
}

// Pass 1: one team of P/16 threads per (slice, n2): gather s[(n1 R + n2 P) mod Q]
// for n1 < P (de-precoded and divided, h = y conj(z) conj(a) / |a|^2), run
// the P-point FFT, write Z[slice][k1][n2].
template <int P>
__global__ void __launch_bounds__(K5Shape<P>::BLOCK) k5g_sft_pass1(K5gArgs a) {
  using C = K5Shape<P>;
  constexpr int T = C::T;
  __shared__ float2 lds_all[C::TEAMS * LdsSize<P>::value];
  const int team = threadIdx.x / T;
  const int t = threadIdx.x - team * T;
  const int gt = blockIdx.x * C::TEAMS + team;
  const bool active = gt < a.total * a.R;
  const int gc = active ? gt : 0;
  const int slice = gc / a.R;
  const int n2 = gc - slice * a.R;
  const int f = slice / (3 * a.n_dirs);
  const int rem = slice - f * 3 * a.n_dirs;
  const int dir = rem / 3;
  const int off = rem - dir * 3;                          // offsets (0,0), (1,0), (0,1)
  const uint32_t al = (uint32_t)a.dir_a[dir], be = (uint32_t)a.dir_b[dir];
  const uint32_t t1 = off == 1 ? 1u : 0u, t2 = off == 2 ? 1u : 0u;
  const RADAR_GLOBAL float2* y = gptr(a.Y + (int64_t)f * a.frame_stride);
  const RADAR_GLOBAL float2* x = gptr(a.A + (int64_t)f * a.frame_stride);
  float2* lds = lds_all + team * LdsSize<P>::value;

  uint32_t st = 0;
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const uint32_t n1 = (uint32_t)(t + T * e);
    const uint32_t tq = (n1 * (uint32_t)a.R + (uint32_t)n2 * (uint32_t)P) % (uint32_t)a.Q;
    const uint32_t k = (al * tq + t1) % (uint32_t)a.N;    // al < N <= 4096, tq < 2^17: no overflow
    const uint32_t l = (be * tq + t2) % (uint32_t)a.M;
    const int64_t idx = (int64_t)l * a.ld + k;
    const float2 yv = gload2(y + idx);
    const float2 av = gload2(x + idx);
    const float2 hz = a.zc ? cmul(yv, a.zc[k]) : yv;
    const float den = cabs2(av);
    st |= den == 0.0f ? 1u : 0u;
    const float inv = den == 0.0f ? 0.0f : __builtin_amdgcn_rcpf(den);
    v[e] = cscale(cmulc(hz, av), inv);
    st |= (__builtin_isfinite(v[e].x) && __builtin_isfinite(v[e].y)) ? 0u : 2u;
  }
  team_fft<P, 16, false>(v, lds, t, active);
  if (!active) return;
  float2* out = a.Z + (int64_t)slice * a.Q + n2;
#pragma unroll
  for (int e = 0; e < 16; ++e) out[(int64_t)(t + T * e) * a.R] = v[e];
  if (st && a.status) atomicOr(a.status + f, st);
}

// Pass 2: one thread per output (slice, k1, k2): the R-point DFT over n2 of
// Z[slice][k1][.], written to S[slice][m(k1, k2)].
__global__ void __launch_bounds__(256) k5g_sft_pass2(K5gArgs a) {
  __shared__ float2 s_wr[kSftGMaxR];
  for (int i = threadIdx.x; i < a.R; i += blockDim.x) s_wr[i] = a.wr[i];
  __syncthreads();
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= (int64_t)a.total * a.Q) return;
  const int slice = (int)(o / a.Q);
  const int rem = (int)(o - (int64_t)slice * a.Q);
  const int k1 = rem / a.R;
  const int k2 = rem - k1 * a.R;
  const RADAR_GLOBAL float2* z = gptr(a.Z + (int64_t)slice * a.Q + (int64_t)k1 * a.R);
  float2 acc = make_float2(0.0f, 0.0f);
  int x = 0;  // n2 k2 mod R
  for (int n2 = 0; n2 < a.R; ++n2) {
    const float2 w = s_wr[x];
    const float2 zv = gload2(z + n2);
    acc.x = fmaf(zv.x, w.x, fmaf(-zv.y, w.y, acc.x));
    acc.y = fmaf(zv.x, w.y, fmaf(zv.y, w.x, acc.y));
    x += k2;
    if (x >= a.R) x -= a.R;
  }
  const int64_t m = ((int64_t)k1 * a.R * a.r_inv + (int64_t)k2 * a.P * a.p_inv) % a.Q;
  a.S[(int64_t)slice * a.Q + m] = acc;
}

struct K6gArgs {
  const float2* S;     // [F][I][3][Q]
  radar_peak* peaks;   // [F][k]
  int32_t* n_peaks;    // [F]
  int N, M, Q, n_dirs, k;
  float nm_over_q;     // N M / Q = gcd(N, M): c = S0 * gcd
  float thr_factor;    // -ln(pfa) / ln 2
  float tol;
  float floor_rel;     // numerically empty bins: power <= floor_rel * raw max
  int dir_a[kSftMaxDirs], dir_b[kSftMaxDirs];
};

__device__ __forceinline__ int sftg_bin(int k1, int k2, int al, int be, int N, int M, int Q) {
  return (int)(((int64_t)al * k1 * (Q / N) + (int64_t)be * k2 * (Q / M)) % Q);
}

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t* red) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t r = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += red[i];
  __syncthreads();
  return r;
}

// The element of ascending rank `rank` among the values key(i) of the
// elements with take(i), i < n, by radix selection over the key's bits
// (digits of DIG bits from the top, NB bits in all): one counting pass per
// digit into an LDS histogram, then the block locates the digit's bucket.
template <int NB, int DIG, class Key, class Take>
__device__ uint64_t block_radix_select(int n, uint64_t rank, const Key& key, const Take& take, uint32_t* hist,
                                       uint32_t* red, uint64_t* s_bcast) {
  constexpr int H = 1 << DIG;
  uint64_t prefix = 0, mask = 0;
  for (int shift = NB - DIG; shift > -DIG; shift -= DIG) {
    const int sh = shift < 0 ? 0 : shift;
    const int bits = shift < 0 ? DIG + shift : DIG;
    const uint64_t dmask = ((uint64_t)1 << bits) - 1;
    for (int i = threadIdx.x; i < H; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      if (!take(i)) continue;
      const uint64_t kv = key(i);
      if ((kv & mask) == prefix) atomicAdd(&hist[(kv >> sh) & dmask], 1u);
    }
    __syncthreads();
    // exclusive scan of the histogram over the block, each thread owning a
    // run of buckets; the thread whose run holds the rank names the bucket
    const int per = (H + (int)blockDim.x - 1) / (int)blockDim.x;
    const int b0 = threadIdx.x * per;
    uint32_t mine = 0;
    for (int b = b0; b < b0 + per && b < H; ++b) mine += hist[b];
    uint32_t incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t up = __shfl_up(incl, o);
      if ((threadIdx.x & 63) >= o) incl += up;
    }
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) before += red[w];
    uint64_t cum = before + incl - mine;
    if (rank >= cum && rank < cum + mine) {
      for (int b = b0; b < b0 + per && b < H; ++b) {
        if (rank < cum + hist[b]) {
          s_bcast[0] = (uint64_t)b;
          s_bcast[1] = rank - cum;
          break;
        }
        cum += hist[b];
      }
    }
    __syncthreads();
    prefix |= s_bcast[0] << sh;
    mask |= dmask << sh;
    rank = s_bcast[1];
    __syncthreads();
  }
  return prefix;
}

// One 1024-thread work-group per frame.
__global__ void __launch_bounds__(kSftDecodeThreads) k6g_sft_decode(K6gArgs a) {
  __shared__ uint32_t s_bits[kSftGMaxQ / 32];         // bins with a peel correction
  __shared__ int s_pbin[kSftMaxK];
  __shared__ float2 s_pcorr[3][kSftMaxK];
  __shared__ int s_npeel;
  __shared__ uint32_t s_hist[2048];
  __shared__ uint64_t s_key[kSftGCap];
  __shared__ int32_t s_dec[kSftGCap];
  __shared__ int s_fk1[kSftMaxK], s_fk2[kSftMaxK];
  __shared__ float2 s_fc[kSftMaxK];
  __shared__ int s_count, s_ng, s_more;
  __shared__ uint32_t s_red[kSftDecodeThreads / 64];
  __shared__ float s_redf[kSftDecodeThreads / 64];
  __shared__ uint64_t s_bc[2];
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int N = a.N, M = a.M, Q = a.Q;
  if (tid == 0) s_count = 0;

  for (int dir = 0; dir < a.n_dirs; ++dir) {
    __syncthreads();
    const int count0 = s_count;
    if (count0 >= a.k) break;
    const int al = a.dir_a[dir], be = a.dir_b[dir];
    const RADAR_GLOBAL float2* src = gptr(a.S + ((int64_t)f * a.n_dirs + dir) * 3 * Q);
    float mx = 0.0f;
    for (int i = tid; i < Q; i += kSftDecodeThreads) mx = fmaxf(mx, cabs2(gload2(src + i)));
    const float floor_p = a.floor_rel * block_max_f32(mx, s_redf);
    // the peel: per bin, the sum of the known components' contributions
    for (int i = tid; i < kSftGMaxQ / 32; i += kSftDecodeThreads) s_bits[i] = 0;
    __syncthreads();
    if (tid == 0) {
      int np = 0;
      for (int j = 0; j < count0; ++j) {
        const int k1 = s_fk1[j], k2 = s_fk2[j];
        const int mb = sftg_bin(k1, k2, al, be, N, M, Q);
        int e = 0;
        while (e < np && s_pbin[e] != mb) ++e;
        if (e == np) {
          s_pbin[np] = mb;
          s_pcorr[0][np] = s_pcorr[1][np] = s_pcorr[2][np] = make_float2(0.0f, 0.0f);
          s_bits[mb >> 5] |= 1u << (mb & 31);
          ++np;
        }
        // (Q/(N M)) c exp(+2 pi i (k1 tau1/N + k2 tau2/M)) at offsets (0,0), (1,0), (0,1)
        const float2 c = cscale(s_fc[j], 1.0f / a.nm_over_q);
        double sn, cs;
        sincospi(2.0 * (double)k1 / (double)N, &sn, &cs);
        const float2 p1 = make_float2((float)cs, (float)sn);
        sincospi(2.0 * (double)k2 / (double)M, &sn, &cs);
        const float2 p2 = make_float2((float)cs, (float)sn);
        s_pcorr[0][e] = cadd(s_pcorr[0][e], c);
        s_pcorr[1][e] = cadd(s_pcorr[1][e], cmul(c, p1));
        s_pcorr[2][e] = cadd(s_pcorr[2][e], cmul(c, p2));
      }
      s_npeel = np;
    }
    __syncthreads();
    auto val = [&](int t, int m) {
      float2 v = gload2(src + (int64_t)t * Q + m);
      if (s_bits[m >> 5] & (1u << (m & 31))) {
        int e = 0;
        while (s_pbin[e] != m) ++e;
        v = csub(v, s_pcorr[t][e]);
      }
      return v;
    };
    // median of |S0|^2 (mean of the two central values, Q even) and the threshold
    auto pkey = [&](int i) { return (uint64_t)ord_bits(cabs2(val(0, i))); };
    auto all = [](int) { return true; };
    const float p_lo = ord_value((uint32_t)block_radix_select<32, 11>(Q, (uint64_t)(Q / 2 - 1), pkey, all, s_hist,
                                                                      s_red, s_bc));
    const float p_hi = ord_value((uint32_t)block_radix_select<32, 11>(Q, (uint64_t)(Q / 2), pkey, all, s_hist,
                                                                      s_red, s_bc));
    const float theta2 = a.thr_factor * (0.5f * (p_hi + p_lo));
    // the candidates, in rounds of at most kSftGCap in descending key order
    uint64_t last = ~0ull;  // exclusive upper bound of this round's keys
    auto ckey = [&](int i) {
      const float p = cabs2(val(0, i));
      return (p >= theta2 && p > floor_p) ? make_key(ord_bits(p), (uint32_t)i) : 0ull;
    };
    while (true) {
      uint32_t mine = 0;
      for (int i = tid; i < Q; i += kSftDecodeThreads) {
        const uint64_t kv = ckey(i);
        mine += (kv != 0 && kv < last) ? 1u : 0u;
      }
      const uint32_t n = block_sum_u32(mine, s_red);
      if (n == 0) break;
      uint64_t lo = 1;  // inclusive lower bound of this round's keys
      if (n > (uint32_t)kSftGCap) {
        auto take = [&](int i) {
          const uint64_t kv = ckey(i);
          return kv != 0 && kv < last;
        };
        // the kSftGCap-th largest key: ascending rank n - kSftGCap
        lo = block_radix_select<64, 8>(Q, (uint64_t)(n - kSftGCap), ckey, take, s_hist, s_red, s_bc);
      }
      if (tid == 0) s_ng = 0;
      __syncthreads();
      for (int i = tid; i < Q; i += kSftDecodeThreads) {
        const uint64_t kv = ckey(i);
        if (kv != 0 && kv < last && kv >= lo) s_key[atomicAdd(&s_ng, 1)] = kv;
      }
      __syncthreads();
      const int ng = s_ng;
      int np2 = 2;
      while (np2 < ng) np2 <<= 1;
      for (int i = ng + tid; i < np2; i += kSftDecodeThreads) s_key[i] = 0;
      bitonic_sort_desc(s_key, np2);
      // test and decode every gathered bin
      for (int j = tid; j < np2; j += kSftDecodeThreads) {
        int dec = -2;
        if (j < ng) {
          dec = -1;
          const int mb = (int)(0xFFFFFFFFu - (uint32_t)s_key[j]);
          const float2 s0 = val(0, mb), s1 = val(1, mb), s2 = val(2, mb);
          const float q0 = cabs2(s0);
          const float r1 = sqrtf(cabs2(s1) / q0), r2 = sqrtf(cabs2(s2) / q0);
          if (fabsf(r1 - 1.0f) <= a.tol && fabsf(r2 - 1.0f) <= a.tol) {
            const float2 c1 = cmulc(s1, s0), c2 = cmulc(s2, s0);  // arg(S1/S0), arg(S2/S0)
            constexpr float kInv2Pi = 0.15915494309189535f;
            int k1 = (int)rintf((float)N * atan2f(c1.y, c1.x) * kInv2Pi) % N;
            int k2 = (int)rintf((float)M * atan2f(c2.y, c2.x) * kInv2Pi) % M;
            k1 += k1 < 0 ? N : 0;
            k2 += k2 < 0 ? M : 0;
            if (sftg_bin(k1, k2, al, be, N, M, Q) == mb) dec = k1 | (k2 << 16);
          }
        }
        s_dec[j] = dec;
      }
      __syncthreads();
      // merge in sorted order (one wavefront; lane q owns found slot q)
      if (tid < 64) {
        int count = s_count;
        bool stop = false;
        for (int j0 = 0; j0 < ng && !stop; j0 += 64) {
          const int j = j0 + tid;
          const int dec = j < ng ? s_dec[j] : -2;
          uint64_t acc = __ballot(dec >= 0);
          while (acc) {
            const int b = __builtin_ctzll(acc);
            acc &= acc - 1;
            const int d = __shfl(dec, b);
            const int k1 = d & 0xFFFF, k2 = d >> 16;
            const int mb = (int)(0xFFFFFFFFu - (uint32_t)s_key[j0 + b]);
            const float2 c = cscale(val(0, mb), a.nm_over_q);
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
        if (tid == 0) {
          s_count = count;
          s_more = (!stop && n > (uint32_t)kSftGCap) ? 1 : 0;
        }
      }
      __syncthreads();
      if (!s_more) break;
      last = s_key[ng - 1];
      __syncthreads();
    }
  }
  __syncthreads();
  // rank by (p descending, flat index ascending) and write the detections
  const int count = s_count;
  if (tid < count) {
    const float inv_nm = 1.0f / ((float)N * (float)M);
    auto cell = [&](int q, float& p) {
      p = cabs2(s_fc[q]) * inv_nm;
      const int k1 = s_fk1[q], k2 = s_fk2[q];
      const int s = k2 < M / 2 ? k2 : k2 - M;
      const int r = (N - k1) % N;
      return make_key(ord_bits(p), (uint32_t)(s + M / 2) * (uint32_t)N + (uint32_t)r);
    };
    float p;
    const uint64_t key = cell(tid, p);
    int rank = 0;
    for (int q = 0; q < count; ++q) {
      float qp;
      rank += cell(q, qp) > key ? 1 : 0;
    }
    const int k1 = s_fk1[tid], k2 = s_fk2[tid];
    radar_peak pk;
    pk.s = k2 < M / 2 ? k2 : k2 - M;
    pk.r = (N - k1) % N;
    pk.p = p;
    pk.s_off = 0.0f;
    pk.r_off = 0.0f;
    a.peaks[(int64_t)f * a.k + rank] = pk;
  }
  if (tid == 0) a.n_peaks[f] = count;
}

}  // namespace radar
