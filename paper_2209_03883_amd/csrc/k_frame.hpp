// The three transform kernels of the receive path, in "tap-first" order.
//
// Every k-axis (subcarrier) operation of the path commutes with every l-axis
// (symbol) operation and the window is separable, so the periodogram of
// Eq. 17 can be formed as
//   K1  per symbol l:  taps  t_l = w_l/N * IDFT_N(Y_l conj(z) / A_l), kept for n < N_cp
//                      (ZC de-precoding Sec. III-B, Eq. 16, Eq. 20-21)
//   K2  per tap n:     U[s][n] = sum_l t_l[n] e^{-2 pi i l s/M'}          (Doppler DFT of Eq. 17)
//   K3  per Doppler s: X = DFT_N(U[s]) (Eq. 22), G[r] = sum_k w_k X_k e^{+2 pi i k r/N'},
//                      P[s][r] = |G[r]|^2 / (N M)                          (range DFT of Eq. 17)
// Only the N_cp taps cross between the symbol pass and the subcarrier pass.
#pragma once

#include "fft.hpp"

namespace radar {

constexpr int kBlock = 256;  // threads per work-group of K1/K2/K3

struct K1Args {
  const float2* Y;        // frames, symbol-major, element (l,k) at l*ld + k
  const float2* A;        // known transmitted symbols (same layout); unused if from_h
  int64_t ld;
  int64_t frame_stride;   // elements between frames of Y / A
  float2* taps;           // [F][M][n_cp]
  uint32_t* status;       // [F] or null
  int M, n_cp;
  int zc_on;              // apply conj(z_k)
  uint32_t zc_root, zc_shift;  // reduced modulo 2N (two's complement for negative shifts)
  int window;
  int from_h;             // input already is the LS estimate H
  int tw_shift_2n;        // twiddle shift for length 2N
  int tw_shift_m;         // twiddle shift for length M
  float inv_n;            // 1/N
};

// K1: one team per OFDM symbol.
template <int N>
__global__ void __launch_bounds__(kBlock) k1_taps(K1Args a) {
  constexpr int T = N / 16;
  constexpr int TEAMS = kBlock / T;
  __shared__ float2 lds_all[TEAMS * LdsSize<N>::value];
  const int team = threadIdx.x / T;
  const int t = threadIdx.x - team * T;
  const int f = blockIdx.y;
  const int l = blockIdx.x * TEAMS + team;
  const bool active = l < a.M;
  const int lc = active ? l : 0;
  float2* lds = lds_all + team * LdsSize<N>::value;

  const float2* y = a.Y + f * a.frame_stride + lc * a.ld;
  const float2* x = a.A + f * a.frame_stride + lc * a.ld;
  uint32_t st = 0;
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int k = t + T * e;
    float2 h = y[k];
    if (!a.from_h) {
      if (a.zc_on) {
        // z_k = exp(+i pi m_k / N) with m_k = root*(k^2 + 2 q k) mod 2N (Eq. 23, even N);
        // 2N divides 2^32, so unsigned wrap-around keeps m_k exact.
        const uint32_t uk = (uint32_t)k;
        const uint32_t m = (a.zc_root * (uk * uk + 2u * a.zc_shift * uk)) & (uint32_t)(2 * N - 1);
        h = cmul(h, twiddle((int)m, a.tw_shift_2n));  // y * conj(z_k)
      }
      const float2 s = x[k];
      const float den = cabs2(s);
      if (den == 0.0f) {
        st |= 1u;
        h = make_float2(0.0f, 0.0f);
      } else {
        h = cscale(cmulc(h, s), 1.0f / den);        // y conj(z) conj(a) / |a|^2
      }
    }
    if (!__builtin_isfinite(h.x) || !__builtin_isfinite(h.y)) st |= 2u;
    v[e] = h;
  }
  team_fft<N, true>(v, lds, t);
  if (!active) return;
  const float scale = window_value(a.window, l, a.tw_shift_m) * a.inv_n;
  float2* out = a.taps + ((int64_t)f * a.M + l) * a.n_cp;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int n = t + T * e;
    if (n < a.n_cp) out[n] = cscale(v[e], scale);
  }
  if (st && a.status) atomicOr(a.status + f, st);
}

struct K2Args {
  const float2* taps;     // [F][M][n_cp]
  float2* U;              // [F][M'][n_cp], row = fftshifted Doppler index
  int M, m_pad, n_cp;
  int fm;                 // M'/M
  int tw_shift_mp;        // twiddle shift for length M'
};

// K2: one team per DFT-CE tap; M'-point Doppler DFT with M non-zero inputs,
// computed as M'/M twiddled M-point FFTs.
template <int M>
__global__ void __launch_bounds__(kBlock) k2_doppler(K2Args a) {
  constexpr int T = M / 16;
  constexpr int TEAMS = kBlock / T;
  __shared__ float2 lds_all[TEAMS * LdsSize<M>::value];
  const int team = threadIdx.x / T;
  const int t = threadIdx.x - team * T;
  const int f = blockIdx.y;
  const int n = blockIdx.x * TEAMS + team;
  const bool active = n < a.n_cp;
  float2* lds = lds_all + team * LdsSize<M>::value;

  const float2* in = a.taps + (int64_t)f * M * a.n_cp + (active ? n : 0);
  float2 x[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) x[e] = in[(int64_t)(t + T * e) * a.n_cp];
  float2* out = a.U + (int64_t)f * a.m_pad * a.n_cp + n;
  const int half = a.m_pad >> 1;
  for (int b = 0; b < a.fm; ++b) {
    float2 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int l = t + T * e;
      v[e] = b == 0 ? x[e] : cmul(x[e], twiddle(l * b, a.tw_shift_mp));
    }
    team_fft<M, false>(v, lds, t);
    if (active) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int su = a.fm * (t + T * e) + b;          // unsigned Doppler index
        const int row = (su + half) & (a.m_pad - 1);    // fftshift
        out[(int64_t)row * a.n_cp] = v[e];
      }
    }
  }
}

struct K3Args {
  const float2* U;        // [F][M'][n_cp]
  float* P;               // frame f at P + f*p_stride, [M'][N']
  int64_t p_stride;
  int m_pad, n_pad, n_cp;
  int window;
  int tw_shift_n;         // twiddle shift for length N
  int tw_shift_np;        // twiddle shift for length N'
  float scale;            // 1/(N M)
};

template <int F2>
__device__ __forceinline__ void store_row_chunk(float* dst, const float (&p)[F2]) {
  if constexpr (F2 == 1) {
    dst[0] = p[0];
  } else if constexpr (F2 == 2) {
    *reinterpret_cast<float2*>(dst) = make_float2(p[0], p[1]);
  } else {
#pragma unroll
    for (int i = 0; i < F2; i += 4)
      *reinterpret_cast<float4*>(dst + i) = make_float4(p[i], p[i + 1], p[i + 2], p[i + 3]);
  }
}

// K3: one team per Doppler row; DFT_N back from the taps, range window, and
// the N'-point range IDFT as F2 = N'/N twiddled N-point inverse FFTs.
template <int N, int F2>
__global__ void __launch_bounds__(kBlock) k3_range_power(K3Args a) {
  constexpr int T = N / 16;
  constexpr int TEAMS = kBlock / T;
  __shared__ float2 lds_all[TEAMS * LdsSize<N>::value];
  const int team = threadIdx.x / T;
  const int t = threadIdx.x - team * T;
  const int f = blockIdx.y;
  const int row = blockIdx.x * TEAMS + team;
  const bool active = row < a.m_pad;
  float2* lds = lds_all + team * LdsSize<N>::value;

  const float2* in = a.U + ((int64_t)f * a.m_pad + (active ? row : 0)) * a.n_cp;
  float2 X[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int k = t + T * e;
    X[e] = k < a.n_cp ? in[k] : make_float2(0.0f, 0.0f);
  }
  team_fft<N, false>(X, lds, t);
#pragma unroll
  for (int e = 0; e < 16; ++e) X[e] = cscale(X[e], window_value(a.window, t + T * e, a.tw_shift_n));

  float pw[16][F2];
#pragma unroll
  for (int b2 = 0; b2 < F2; ++b2) {
    float2 g[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int k = t + T * e;
      g[e] = b2 == 0 ? X[e] : cmulc(X[e], twiddle(k * b2, a.tw_shift_np));  // X e^{+2 pi i k b2/N'}
    }
    team_fft<N, true>(g, lds, t);
#pragma unroll
    for (int e = 0; e < 16; ++e) pw[e][b2] = cabs2(g[e]) * a.scale;
  }
  if (!active) return;
  float* dst = a.P + (int64_t)f * a.p_stride + (int64_t)row * a.n_pad;
#pragma unroll
  for (int e = 0; e < 16; ++e) store_row_chunk<F2>(dst + F2 * (t + T * e), pw[e]);
}

// Clears the per-frame status and peak-count words (a fill kernel rather than
// a memset, so the sequence stays safe inside captured graphs).
__global__ void k0_clear(uint32_t* status, int32_t* n_peaks, int n_frames) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_frames) {
    if (status) status[i] = 0u;
    if (n_peaks) n_peaks[i] = 0;
  }
}

}  // namespace radar
