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
#include "mfma_dft.hpp"

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
  uint32_t zc_root, zc_shift;  // reduced modulo 2N; root 0 = no precoding
  int window;
  int from_h;             // input already is the LS estimate H
  float inv_n;            // 1/N
  const FrameRef* refs;   // per-frame Y, A, status (batch jobs), or null: base + f * frame_stride
  float* inv_sum;         // [F][M] sum_k 1/|a_{l,k}|^2 per symbol (threshold detection), or null
  const float* tap_w;     // [n_cp] LMMSE weights of the kept taps, or null (plain DFT-CE)
};

// Sum over the T threads of one team (T a power of two; teams inside one
// wave when T <= 64, else whole work-group rows of T threads with LDS `red`
// of T/64 floats per team).  Every thread of the team gets the sum.
template <int T>
__device__ __forceinline__ float team_sum(float v, float* red, int team, int t) {
#pragma unroll
  for (int m = (T < 64 ? T : 64) / 2; m > 0; m >>= 1) v += __shfl_xor(v, m);
  if constexpr (T > 64) {
    if ((t & 63) == 0) red[team * (T / 64) + (t >> 6)] = v;
    __syncthreads();
    v = 0.0f;
#pragma unroll
    for (int w = 0; w < T / 64; ++w) v += red[team * (T / 64) + w];
    __syncthreads();
  }
  return v;
}

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

  const RADAR_GLOBAL float2* y = gptr(a.refs ? a.refs[f].Y : a.Y + f * a.frame_stride) + lc * a.ld;
  const RADAR_GLOBAL float2* x = gptr(a.refs ? a.refs[f].A : a.A + f * a.frame_stride) + lc * a.ld;
  uint32_t st = 0;
  float isum = 0.0f;
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = gload2(y + t + T * e);
  if (!a.from_h) {
    float2 s[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) s[e] = gload2(x + t + T * e);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int k = t + T * e;
      // z_k = exp(+i pi m_k / N) with m_k = root*(k^2 + 2 q k) mod 2N (Eq. 23, even N);
      // 2N divides 2^32, so unsigned wrap-around keeps m_k exact.  Without
      // precoding root = 0 and the factor is exactly 1.
      const uint32_t uk = (uint32_t)k;
      const uint32_t m = (a.zc_root * (uk * uk + 2u * a.zc_shift * uk)) & (uint32_t)(2 * N - 1);
      const float2 h = cmul(v[e], twiddle_split(2 * N, (int)m));  // y * conj(z_k)
      const float den = cabs2(s[e]);
      st |= den == 0.0f ? 1u : 0u;
      const float inv = den == 0.0f ? 0.0f : __builtin_amdgcn_rcpf(den);
      isum += inv;
      v[e] = cscale(cmulc(h, s[e]), inv);            // y conj(z) conj(a) / |a|^2
    }
    if (a.inv_sum) {
      __shared__ float red[T > 64 ? TEAMS * (T / 64) : 1];
      isum = team_sum<T>(isum, red, team, t);
      if (active && t == 0) a.inv_sum[(int64_t)f * a.M + l] = isum;
    }
  }
#pragma unroll
  for (int e = 0; e < 16; ++e)
    st |= (__builtin_isfinite(v[e].x) && __builtin_isfinite(v[e].y)) ? 0u : 2u;
  team_fft<N, 16, true>(v, lds, t);
  if (!active) return;
  const float scale = window_value(a.window, l, a.M) * a.inv_n;
  float2* out = a.taps + ((int64_t)f * a.M + l) * a.n_cp;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int n = t + T * e;
    if (n < a.n_cp) out[n] = cscale(v[e], a.tap_w ? scale * a.tap_w[n] : scale);
  }
  if (st) {
    uint32_t* sp = a.refs ? a.refs[f].status : (a.status ? a.status + f : nullptr);
    if (sp) atomicOr(sp, st);
  }
}


// K1, persistent form (N <= 1024): each work-group copies the ZC phase table
// W_{2N}^m (m < 2N) and the twiddle blocks of the inverse FFT plan into LDS
// once; its waves then loop over OFDM symbols, one symbol per wave.
template <int N>
struct K1p {
  static constexpr int T = N / 16;
  static constexpr int ROWS = 64 / T;                      // symbols per wave per pass
  static constexpr int WAVES = 8;
  static constexpr int BLOCK = 64 * WAVES;
  static constexpr int ZC = 0;                             // W_{2N}^m, m < 2N
  static constexpr int INV = 2 * N;
  static constexpr int TAB = INV + PlanTable<N, 16, 1>::size();
  static constexpr int EXCH = LdsSize<N>::value;
  using Inv = PlanLayout<N, INV, 1>;
};

template <int N>
__global__ void __launch_bounds__(K1p<N>::BLOCK) k1_taps_p(K1Args a, int total_groups) {
  using C = K1p<N>;
  constexpr int T = C::T;
  __shared__ float2 tab[C::TAB];
  __shared__ float2 xch[C::WAVES][C::ROWS][C::EXCH];
  for (int i = threadIdx.x; i < 2 * N; i += C::BLOCK) tab[C::ZC + i] = g_radar_tw[(unsigned)(2 * N + i)];
  copy_plan_twiddles<N, 16, 1>(tab + C::INV, threadIdx.x, C::BLOCK);
  __syncthreads();
  const TwLds<typename C::Inv> tw_inv{tab};
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane / T;
  const int t = lane - g * T;
  float2* lds = xch[wave][g];

  for (int grp = blockIdx.x * C::WAVES + wave; grp < total_groups; grp += gridDim.x * C::WAVES) {
    const int gsym = grp * C::ROWS + g;                     // symbol over all frames
    const int f = gsym / a.M;
    const int l = gsym - f * a.M;
    const RADAR_GLOBAL float2* y = gptr(a.refs ? a.refs[f].Y : a.Y + f * a.frame_stride) + l * a.ld;
    const RADAR_GLOBAL float2* x = gptr(a.refs ? a.refs[f].A : a.A + f * a.frame_stride) + l * a.ld;
    uint32_t st = 0;
    float isum = 0.0f;
    float2 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = gload2(y + t + T * e);
    if (!a.from_h) {
      float2 sv[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) sv[e] = gload2(x + t + T * e);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int k = t + T * e;
        // z_k = exp(+i pi m_k / N), m_k = root*(k^2 + 2 q k) mod 2N (Eq. 23, even N);
        // without precoding root = 0, so m_k = 0 and the factor is exactly 1
        const uint32_t uk = (uint32_t)k;
        const uint32_t m = (a.zc_root * (uk * uk + 2u * a.zc_shift * uk)) & (uint32_t)(2 * N - 1);
        const float2 h = cmul(v[e], tab[C::ZC + m]);  // y * conj(z_k)
        const float den = cabs2(sv[e]);
        st |= den == 0.0f ? 1u : 0u;
        const float inv = den == 0.0f ? 0.0f : __builtin_amdgcn_rcpf(den);
        isum += inv;
        v[e] = cscale(cmulc(h, sv[e]), inv);          // y conj(z) conj(a) / |a|^2
      }
      if (a.inv_sum) {
        isum = team_sum<T>(isum, nullptr, 0, t);
        if (t == 0) a.inv_sum[gsym] = isum;
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e)
      st |= (__builtin_isfinite(v[e].x) && __builtin_isfinite(v[e].y)) ? 0u : 2u;
    fft_stages<N, 16, 1, true>(v, lds, t, true, tw_inv);
    const float scale = window_value(a.window, l, a.M) * a.inv_n;
    float2* out = a.taps + (int64_t)gsym * a.n_cp;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int n = t + T * e;
      if (n < a.n_cp) out[n] = cscale(v[e], a.tap_w ? scale * a.tap_w[n] : scale);
    }
    if (st) {
      uint32_t* sp = a.refs ? a.refs[f].status : (a.status ? a.status + f : nullptr);
      if (sp) atomicOr(sp, st);
    }
  }
}

struct K2Args {
  const float2* taps;     // [F][M][n_cp]
  float2* U;              // [F][M'][n_cp], row = fftshifted Doppler index
  int M, m_pad, n_cp;
  int fm;                 // M'/M
  int ph_off;             // phase-section offset of W_{M'}^{l b} (layout [b][l]), or -1: power section
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
      const float2 w = a.ph_off >= 0 ? g_radar_tw[(unsigned)(a.ph_off + b * M + l)] : twiddle(a.m_pad, l * b);
      v[e] = b == 0 ? x[e] : cmul(x[e], w);
    }
    team_fft<M, 16, false>(v, lds, t);
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


// K2, tiled: one team per (tap, Doppler sub-transform b); a work-group covers
// TW adjacent taps for one b.  The taps come in as rows of TW contiguous
// elements through an LDS tile, and the results leave the same way, so every
// global access is a contiguous row segment.
//   U[M'/M * s1 + b][n] = FFT_M(t_l[n] W_{M'}^{l b})[s1]   (fftshifted row index)
template <int M, int TW>
struct K2Tile {
  static constexpr int T = M / 16;
  static constexpr int BLOCK = TW * T;
  static constexpr int EXCH = LdsSize<M>::value;
  static constexpr int LD = TW + 1;  // padded tile row (limits bank conflicts)
  static constexpr int SH = TW * EXCH > M * LD ? TW * EXCH : M * LD;
  // the FFT plan's twiddles in LDS where they fit beside the tile (else they
  // are read from the global table)
  static constexpr int PLAN = PlanTable<M, 16, 1>::size();
  static constexpr bool kLdsTw = (SH + PLAN) * 8 <= 150 * 1024;
  static constexpr int TWN = kLdsTw && PLAN > 0 ? PLAN : 1;
  using Plan = PlanLayout<M, 0, 1>;
};

// K2 runs persistent in the FP32 form; the matrix-core forms hold their DFT
// fragments in registers throughout and launch one work-group per item.
template <Prec PR>
struct K2Persistent {
  static constexpr bool value = PR == Prec::FP32;
};

template <int M, int TW, Prec PR = Prec::FP32>
__global__ void __launch_bounds__((K2Tile<M, TW>::BLOCK)) k2_doppler_tiled(K2Args a, int n_tiles, int total) {
  using C = K2Tile<M, TW>;
  typename DftFor<PR>::type df;
  df.init();
  constexpr int T = C::T, BLOCK = C::BLOCK, LD = C::LD;
  __shared__ float2 sh[C::SH];
  __shared__ float2 twtab[C::TWN];
  if constexpr (C::kLdsTw) copy_plan_twiddles<M, 16, 1>(twtab, threadIdx.x, BLOCK);  // ordered by the tile's barrier
  const int team = threadIdx.x / T;
  const int t0 = threadIdx.x - team * T;
  const int half = a.m_pad >> 1;

  // one (tile, b, frame) item, tile fastest
  auto run = [&](int item) {
    // the team lane, opaque to the optimiser (an empty asm statement emits
    // no instruction) and masked back to its range: the per-element LDS
    // addresses are formed again per item instead of held in registers
    int t = t0;
    asm volatile("" : "+v"(t));
    t &= T - 1;
    const int tile = item % n_tiles;
    const int rest = item / n_tiles;
    const int b = rest % a.fm;
    const int f = rest / a.fm;
    const int n0 = tile * TW;
    const int ntap = min(TW, a.n_cp - n0);

    // tile of taps [l][n0 .. n0+TW).  Up to M = 1024 each thread issues its
    // loads eight at a time before the LDS stores: a load per loop iteration
    // with a wait before each store serialises the memory latency.  The
    // ragged last tile clamps its column and stores zeros there, so every
    // load is unconditional and in bounds.  The longest transforms keep the
    // plain loop (their FFT leaves no registers for the batch).
    static_assert(M * TW == 16 * BLOCK, "16 tile elements per thread");
    constexpr bool kBatched = M <= 1024;
    const float2* in = a.taps + (int64_t)f * M * a.n_cp + n0;
    if constexpr (kBatched) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float2 tv[8];
#pragma unroll
        for (int it = 0; it < 8; ++it) {
          const int i = threadIdx.x + (8 * h + it) * BLOCK;
          const int l = i / TW, c = i - l * TW;
          tv[it] = in[(int64_t)l * a.n_cp + (c < ntap ? c : ntap - 1)];
        }
        // the previous item's reads of the tile are done before it is refilled
        if (h == 0) __syncthreads();
#pragma unroll
        for (int it = 0; it < 8; ++it) {
          const int i = threadIdx.x + (8 * h + it) * BLOCK;
          const int l = i / TW, c = i - l * TW;
          sh[l * LD + c] = c < ntap ? tv[it] : make_float2(0.0f, 0.0f);
        }
      }
    } else {
      __syncthreads();
      for (int i = threadIdx.x; i < M * TW; i += BLOCK) {
        const int l = i / TW, c = i - l * TW;
        sh[l * LD + c] = c < ntap ? in[(int64_t)l * a.n_cp + c] : make_float2(0.0f, 0.0f);
      }
    }
    __syncthreads();
    float2 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = sh[(t + T * e) * LD + team];
    if (b != 0) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int l = t + T * e;
        const float2 w = a.ph_off >= 0 ? g_radar_tw[(unsigned)(a.ph_off + b * M + l)] : twiddle(a.m_pad, l * b);
        v[e] = cmul(v[e], w);
      }
    }
    __syncthreads();  // the tile is reused as exchange space
    if constexpr (C::kLdsTw)
      fft_stages<M, 16, 1, false>(v, sh + team * C::EXCH, t, true, TwLds<typename C::Plan>{twtab}, df);
    else
      team_fft<M, 16, false>(v, sh + team * C::EXCH, t, true, df);
    __syncthreads();  // every team is done with its exchange region
#pragma unroll
    for (int e = 0; e < 16; ++e) sh[(t + T * e) * LD + team] = v[e];
    __syncthreads();
    float2* out = a.U + (int64_t)f * a.m_pad * a.n_cp + n0;
    for (int i = threadIdx.x; i < M * TW; i += BLOCK) {
      const int s1 = i / TW, c = i - s1 * TW;
      if (c < ntap) {
        const int row = (a.fm * s1 + b + half) & (a.m_pad - 1);
        out[(int64_t)row * a.n_cp + c] = sh[s1 * LD + c];
      }
    }
  };
  if constexpr (K2Persistent<PR>::value) {
    // persistent over the items: a work-group's stores of one item drain
    // while it loads the next
    for (int item = blockIdx.x; item < total; item += gridDim.x) run(item);
  } else {
    run(blockIdx.x);  // one work-group per item (the loop-carried state would spill)
  }
}

struct K3Args {
  const float2* U;        // [F][M'][n_cp]
  float* P;               // frame f at P + f*p_stride, [M'][N']
  int64_t p_stride;
  int m_pad, n_pad, n_cp;
  int window;
  float scale;            // 1/(N M)
  float* rowmax;          // [F][M'] row maxima of P (written by the x4 kernel), or null
  const FrameRef* refs;   // per-frame P (batch jobs), or null: P + f * p_stride
};

template <int F2>
__device__ __forceinline__ void store_row_chunk(RADAR_GLOBAL float* dst, const float (&p)[F2]) {
  if constexpr (F2 == 1) {
    dst[0] = p[0];
  } else if constexpr (F2 == 2) {
    gstore2(dst, p[0], p[1]);
  } else {
#pragma unroll
    for (int i = 0; i < F2; i += 4)
      gstore4(dst + i, p[i], p[i + 1], p[i + 2], p[i + 3]);
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
  team_fft<N, 16, false>(X, lds, t);
#pragma unroll
  for (int e = 0; e < 16; ++e) X[e] = cscale(X[e], window_value(a.window, t + T * e, N));

  float pw[16][F2];
#pragma unroll
  for (int b2 = 0; b2 < F2; ++b2) {
    float2 g[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int k = t + T * e;
      g[e] = b2 == 0 ? X[e] : cmulc(X[e], phase_twiddle<N, F2>(b2, k));  // X e^{+2 pi i k b2/N'}
    }
    team_fft<N, 16, true>(g, lds, t);
#pragma unroll
    for (int e = 0; e < 16; ++e) pw[e][b2] = cabs2(g[e]) * a.scale;
  }
  if (!active) return;
  RADAR_GLOBAL float* dst = gptr(a.refs ? a.refs[f].P : a.P + (int64_t)f * a.p_stride) + (int64_t)row * a.n_pad;
#pragma unroll
  for (int e = 0; e < 16; ++e) store_row_chunk<F2>(dst + F2 * (t + T * e), pw[e]);
}


// ------------------------------------------------------------------------
// K3 for 4x range padding (N' = 4N) and N_cp <= N/4: one work-group row
// group of four teams per Doppler row.
//
//   forward  X[4 k1 + b] = FFT_{N/4}(u_n W_N^{n b})[k1]      (team b; u has
//            only N_cp <= N/4 non-zero taps, so the N-point DFT of Eq. 22
//            splits into four N/4-point transforms)
//   range    G[4 r1 + b] = sum_k w_k X_k e^{+2 pi i k (4 r1 + b)/(4N)}
//            = IFFT_N(w_k X_k e^{+2 pi i k b/(4N)})[r1]      (team b = 1, 2, 3)
//   phase 0  G[4 r1] = N (c * u)[r1] with c = IDFT_N(w): for the cosine
//            windows w_k = a0 - a1 cos(2 pi k/N) this is the 3-tap filter
//            N (a0 u[r1] - a1/2 (u[r1-1] + u[r1+1]))  (team 0)
// The four phases meet in LDS, the row leaves as contiguous float4 stores,
// and the row maximum is reduced on the way out for the peak search.
// ------------------------------------------------------------------------
template <int N>
struct K3x4 {
  static constexpr int T = N / 16;                    // threads per team
  static constexpr int GROUP = 4 * T;                 // threads per Doppler row
  static constexpr int ROWS = GROUP >= 256 ? 1 : 256 / GROUP;
  static constexpr int BLOCK = GROUP * ROWS;
  static constexpr int EXCH = LdsSize<N>::value;      // float2 per team exchange region
  static constexpr int MAIN = 4 * EXCH;               // float2; holds X (N) or the P row (4N floats)
  static constexpr int UBUF = N / 4 + 3;              // u[-1 .. N/4+1]
};

template <int N, Prec PR = Prec::FP32>
__global__ void __launch_bounds__(K3x4<N>::BLOCK) k3_range_power_x4(K3Args a) {
  using C = K3x4<N>;
  typename DftFor<PR>::type df;
  df.init();
  constexpr int T = C::T;
  constexpr int Q = N / 4;
  __shared__ float2 s_main[C::ROWS][C::MAIN];
  __shared__ float2 s_u[C::ROWS][C::UBUF];
  __shared__ float s_max[C::BLOCK / 64];
  const int g = threadIdx.x / C::GROUP;
  const int gi = threadIdx.x - g * C::GROUP;
  const int team = gi / T;
  const int t = gi - team * T;
  const int f = blockIdx.y;
  const int row = blockIdx.x * C::ROWS + g;            // m_pad is a multiple of ROWS
  float2* main = s_main[g];
  float2* ub = s_u[g] + 1;                             // ub[i] = u[i], i in [-1, N/4+1]

  // Doppler-row taps u_n, n < N_cp <= N/4 (GROUP = N/4 threads: one each)
  const float2* in = a.U + ((int64_t)f * a.m_pad + row) * a.n_cp;
  ub[gi] = gi < a.n_cp ? in[gi] : make_float2(0.0f, 0.0f);
  if (gi < 2) ub[gi == 0 ? -1 : Q] = make_float2(0.0f, 0.0f);
  if (gi == 2) ub[Q + 1] = make_float2(0.0f, 0.0f);
  __syncthreads();

  // forward: team b computes X[4 k1 + b], k1 = t + T e
  {
    float2 x[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int n = t + T * e;
      x[e] = team == 0 ? ub[n] : cmul(ub[n], phase_twiddle<Q, 4>(team, n));
    }
    team_fft<Q, 4, false>(x, main + team * C::EXCH, t);
    __syncthreads();  // exchange regions are reused for X below
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 4 * (t + T * e) + team;
      main[k] = cscale(x[e], window_value(a.window, k, N));
    }
  }
  __syncthreads();

  // range phases
  const bool fft_team = team != 0;
  float2 gv[16];
  if (fft_team) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int k = t + T * e;
      gv[e] = cmulc(main[k], phase_twiddle<N, 4>(team, k));  // X_k e^{+2 pi i k b/(4N)}
    }
  }
  __syncthreads();  // X consumed before the exchange regions overwrite it
  team_fft<N, 16, true>(gv, main + team * C::EXCH, t, fft_team, df);
  float p[16];
  if (fft_team) {
#pragma unroll
    for (int e = 0; e < 16; ++e) p[e] = cabs2(gv[e]) * a.scale;
  } else {
    const float2 wc = window_coeffs(a.window);
    const float c0 = (float)N * wc.x, c1 = -0.5f * (float)N * wc.y;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int r1 = t + T * e;
      float2 gz = make_float2(0.0f, 0.0f);
      if (r1 <= Q) {
        gz = cadd(cscale(ub[r1], c0), cscale(cadd(ub[r1 - 1], ub[r1 + 1]), c1));
      } else if (r1 == N - 1) {
        gz = cscale(ub[0], c1);                                      // u[N] = u[0] wraps round
      }
      p[e] = cabs2(gz) * a.scale;
    }
  }
  __syncthreads();  // exchange regions free: assemble the row
  float* prow = reinterpret_cast<float*>(main);
#pragma unroll
  for (int e = 0; e < 16; ++e) prow[4 * (t + T * e) + team] = p[e];
  __syncthreads();

  RADAR_GLOBAL float* dst = gptr(a.refs ? a.refs[f].P : a.P + (int64_t)f * a.p_stride) + (int64_t)row * (4 * N);
  float mx = 0.0f;
#pragma unroll
  for (int i = gi; i < N; i += C::GROUP) {
    const float4 q = reinterpret_cast<const float4*>(prow)[i];
    gstore4(dst + 4 * i, q.x, q.y, q.z, q.w);
    mx = fmaxf(mx, fmaxf(fmaxf(q.x, q.y), fmaxf(q.z, q.w)));
  }
  // row maximum over the GROUP threads of this row
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
  if constexpr (C::GROUP >= 64) {
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (gi == 0) {
      float r = s_max[(g * C::GROUP) >> 6];
      for (int w = 1; w < C::GROUP / 64; ++w) r = fmaxf(r, s_max[((g * C::GROUP) >> 6) + w]);
      a.rowmax[(int64_t)f * a.m_pad + row] = r;
    }
  } else {
    if (gi == 0) a.rowmax[(int64_t)f * a.m_pad + row] = mx;
  }
}

// ------------------------------------------------------------------------
// K3 for 4x range padding and N_cp <= N/4, N <= 1024: persistent waves, one
// wavefront per Doppler row (four rows per wave at N = 256), all four phases
// of the row in sequence.
//   forward  DFT_N of u (N_cp <= N/4 taps): the first radix-4 Stockham stage
//            of a zero-padded input only copies, y[i] = u[i >> 2], so the
//            transform starts at span 4 straight from the taps.
//   phases   b = 1, 2, 3: IFFT_N(w_k X_k e^{+2 pi i k b/(4N)});
//            b = 0: the 3-tap filter N (a0 u[r1] - a1/2 (u[r1-1] + u[r1+1])).
//   output   the four |G|^2 values of each r1 leave in one 16-byte store
//            where two phases can be held in registers (FP32, N >= 512),
//            else as two 8-byte pairs.
// Every twiddle a row needs is the same for all rows, so each work-group
// copies the stage blocks of its two FFT plans and the phase twiddles
// W_{4N}^{k b} (b = 1..3, each times the window w_k) into LDS once, and its
// waves then loop over rows independently: twiddle reads are LDS reads, not
// vector-memory instructions.
// ------------------------------------------------------------------------
template <int N>
struct K3p {
  static constexpr int T = N / 16;
  static constexpr int ROWS = 64 / T;                   // rows per wave per pass
  static constexpr int WAVES = 8;
  static constexpr int BLOCK = 64 * WAVES;
  static constexpr int FWD = 0;                         // forward plan (from span 4)
  static constexpr int INV = PlanTable<N, 16, 4>::size();  // inverse plan (from span 1)
  static constexpr int PH = INV + PlanTable<N, 16, 1>::size();  // w_k W_{4N}^{k b}, b = 1..3
  static constexpr int TAB = PH + 3 * N;
  static constexpr int EXCH = LdsSize<N>::value;
  static constexpr int UBUF = N / 4 + 3;
  using Fwd = PlanLayout<N, FWD, 4>;
  using Inv = PlanLayout<N, INV, 1>;
};

// Phase 0 of the range IDFT (r = 4 r1) without a transform: the windowed
// spectrum's inverse at the native bins is the three-tap filter c0 u[r1] +
// c1 (u[r1-1] + u[r1+1]) of the taps (zero beyond N/4, u[N] = u[0]).
template <int N>
__device__ __forceinline__ float2 phase0_filter(const float2* ub, int r1, float c0, float c1) {
  constexpr int Q = N / 4;
  if (r1 <= Q) return cadd(cscale(ub[r1], c0), cscale(cadd(ub[r1 - 1], ub[r1 + 1]), c1));
  if (r1 == N - 1) return cscale(ub[0], c1);
  return make_float2(0.0f, 0.0f);
}

// Where one range row of P goes: cell i (in r = 4 r1 + b order) and the
// next one, two or four cells.  P is written once and read back only in the
// few rows the peak search scans, so the whole 16-byte groups are stored
// non-temporally: they do not displace the taps and Doppler rows from the
// caches (measured: the range stage 1.5 % faster, the taps and peak stages a
// few per cent).  The 8-byte halves of the two-store order stay ordinary
// stores, which the caches combine into whole lines: streamed past them, the
// halves written at different times made the BF16x3 range stage 1.8x slower.
struct RowToGlobal {
  RADAR_GLOBAL float* dst;
  __device__ __forceinline__ void store4(int i, float a, float b, float c, float d) const {
    __builtin_nontemporal_store(radar_v4{a, b, c, d}, (RADAR_GLOBAL radar_v4*)(dst + i));
  }
  __device__ __forceinline__ void store2(int i, float a, float b) const { gstore2(dst + i, a, b); }
};
// Nowhere: only the row maximum is kept (P not materialised).
struct RowToNowhere {
  __device__ __forceinline__ void store4(int, float, float, float, float) const {}
  __device__ __forceinline__ void store2(int, float, float) const {}
};
// An LDS row (16-byte aligned), or nowhere when null.
struct RowToLds {
  float* row;
  __device__ __forceinline__ void store4(int i, float a, float b, float c, float d) const {
    if (row) *reinterpret_cast<float4*>(row + i) = make_float4(a, b, c, d);
  }
  __device__ __forceinline__ void store2(int i, float a, float b) const {
    if (row) *reinterpret_cast<float2*>(row + i) = make_float2(a, b);
  }
};

// one 16-byte store per four-phase group where holding two phases fits in
// registers (no scratch): measured for the FP32 form at N >= 512
template <int N, Prec PR>
struct K3pOrder {
  static constexpr bool kOneStore = PR == Prec::FP32 && N >= 512;
};

// The range kernel's LDS tables: the stage blocks of its two FFT plans, then
// the phase twiddles W_{4N}^{k b} (b = 1..3) times the window w_k = a0 - a1
// cos(2 pi k/N) times rs = sqrt(1/(N M)): the normalisation applied to the
// transform inputs (the transform is linear), so |G|^2 comes out normalised
// with no multiply per cell.  Returns the phase-0 filter's coefficients
// (c0, c1), which carry rs too.
template <int N>
__device__ __forceinline__ float2 k3p_tables(float2* tab, int window, float scale, int tid, int nthreads) {
  using C = K3p<N>;
  copy_plan_twiddles<N, 16, 4>(tab + C::FWD, tid, nthreads);
  copy_plan_twiddles<N, 16, 1>(tab + C::INV, tid, nthreads);
  const float2 wc = window_coeffs(window);
  const float rs = sqrtf(scale);
  constexpr int poff = phase_offset(ilog2c(N), 2);
  for (int i = tid; i < 3 * N; i += nthreads) {
    const float w = (wc.x - wc.y * g_radar_tw[(unsigned)(N + (i & (N - 1)))].x) * rs;
    tab[C::PH + i] = cscale(g_radar_tw[(unsigned)(poff + N + i)], w);
  }
  return make_float2((float)N * wc.x * rs, -0.5f * (float)N * wc.y * rs);
}

// The taps of one Doppler row held by lane t of its team: u[t + T e], e < 4.
template <int N>
__device__ __forceinline__ void k3p_load_taps(float2 (&uv)[4], const float2* in, int n_cp, int t) {
  constexpr int T = N / 16;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int n = t + T * e;
    uv[e] = in[n < n_cp ? n : 0];
  }
}
// ... into the team's tap buffer ub[0 .. N/4), zero beyond N_cp.  The pads
// ub[-1], ub[N/4], ub[N/4+1] are zeroed once by k3p_zero_pads.
template <int N>
__device__ __forceinline__ void k3p_put_taps(float2* ub, const float2 (&uv)[4], int n_cp, int t) {
  constexpr int T = N / 16;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int n = t + T * e;
    ub[n] = n < n_cp ? uv[e] : make_float2(0.0f, 0.0f);
  }
}
template <int N>
__device__ __forceinline__ void k3p_zero_pads(float2* ub, int t) {
  if (t < 3) ub[t == 0 ? -1 : N / 4 + t - 1] = make_float2(0.0f, 0.0f);
}

// One Doppler row of the range stage by one team of T = N/16 lanes (lane t):
// the taps u (N_cp <= N/4 of them) already in `ub` (LDS, ub[-1 .. N/4+1],
// from k3p_put_taps and k3p_zero_pads), the forward DFT_N, the three phase
// IFFTs and the phase-0 filter, every |G|^2 cell to `sink`.  `next()` runs
// just before the first store: the caller loads the next row's taps into
// registers there and puts them in ub after this returns, so that their wait
// comes after this row's stores in straight-line code and does not include
// them (a vector-memory wait covers every older load and store, and a wait at
// the top of the row loop would be merged with the first row's).  Returns the
// row maximum (in every lane of the team).  The team's LDS exchange region is
// `lds`.
template <int N, Prec PR, class DF, class Sink, class Next>
__device__ __forceinline__ float k3p_row(float2* lds, float2* ub, int t, const float2* tab, float c0, float c1,
                                         const DF& df, const Sink& sink, const Next& next) {
  using C = K3p<N>;
  constexpr int T = C::T;
  constexpr int Q = N / 4;
  static_assert(T % 4 == 0, "the forward load indexes u[(t + T e) / 4] as t/4 + (T/4) e");
  static_assert(Q / T == 4, "four taps per lane");
  const TwLds<typename C::Fwd> tw_fwd{tab};
  const TwLds<typename C::Inv> tw_inv{tab};
  team_sync<64>();

  // forward DFT_N from span 4 (the zero-padded first radix-4 stage only
  // copies): element t + T e takes u[(t + T e) / 4] = u[t/4 + (T/4) e]
  float2 X[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) X[e] = ub[(t >> 2) + (T / 4) * e];
  fft_stages<N, 16, 4, false>(X, lds, t, true, tw_fwd, df);

  float mx = 0.0f;
  if constexpr (K3pOrder<N, PR>::kOneStore) {
    // phases 1, 2, 3 in turn; X dies after the last twiddle product, so
    // holding p1 and p2 through the last transform costs no more registers
    // than X did, and each four-phase group of P leaves in one 16-byte store
    float p1[16], p2[16];
#pragma unroll
    for (int phase = 1; phase <= 3; ++phase) {
      float2 gv[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) gv[e] = cmulc(X[e], tab[C::PH + (phase - 1) * N + t + T * e]);
      fft_stages<N, 16, 1, true>(gv, lds, t, true, tw_inv, df);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const float pv = cabs2(gv[e]);
        if (phase == 1) p1[e] = pv;
        else if (phase == 2) p2[e] = pv;
        else gv[e].x = pv;  // p3
      }
      if (phase == 3) {
        next();
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const float p0 = cabs2(phase0_filter<N>(ub, t + T * e, c0, c1));
          sink.store4(4 * (t + T * e), p0, p1[e], p2[e], gv[e].x);
          mx = fmaxf(fmaxf(fmaxf(fmaxf(mx, p0), p1[e]), p2[e]), gv[e].x);
        }
      }
    }
  } else {
    // phases 2 and 3 leave as one 8-byte store, then phase 1 and phase 0
    float p_first[16];
#pragma unroll
    for (int b = 2; b <= 4; ++b) {
      const int phase = b == 4 ? 1 : b;
      float2 gv[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) gv[e] = cmulc(X[e], tab[C::PH + (phase - 1) * N + t + T * e]);
      fft_stages<N, 16, 1, true>(gv, lds, t, true, tw_inv, df);
      if (phase == 3) {
        next();
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const float p3 = cabs2(gv[e]);
          sink.store2(2 * (2 * (t + T * e) + 1), p_first[e], p3);
          mx = fmaxf(mx, fmaxf(p_first[e], p3));
        }
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) p_first[e] = cabs2(gv[e]);
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const float p0 = cabs2(phase0_filter<N>(ub, t + T * e, c0, c1));
      sink.store2(4 * (t + T * e), p0, p_first[e]);
      mx = fmaxf(mx, fmaxf(p0, p_first[e]));
    }
  }
#pragma unroll
  for (int m = T / 2; m > 0; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
  return mx;
}

// kStore = false: the row maxima only, P not written (the peak search then
// recomputes the few rows it needs).  kRefs: P row pointers from the batch
// job table (a.refs) rather than a.P + f * p_stride; a separate instance, as
// the table load on one path would make the wait for the next row's taps
// cover the previous row's stores on both.
template <int N, Prec PR = Prec::FP32, bool kStore = true, bool kRefs = false>
__global__ void __launch_bounds__(K3p<N>::BLOCK) k3_range_power_x4p(K3Args a, int total_groups) {
  using C = K3p<N>;
  constexpr bool kOneStore = K3pOrder<N, PR>::kOneStore;
  typename DftFor<PR>::type df;
  df.init();
  constexpr int T = C::T;
  // one pool with the twiddle table first: its offsets stay below 64 KiB, so
  // every table read encodes its constant part as the instruction's offset
  static_assert(C::TAB * 8 < 65536, "twiddle table beyond the LDS offset range");
  __shared__ float2 pool[C::TAB + C::WAVES * C::ROWS * (C::EXCH + C::UBUF)];
  float2* const tab = pool;
  auto xch = reinterpret_cast<float2 (*)[C::ROWS][C::EXCH]>(pool + C::TAB);
  auto ubuf = reinterpret_cast<float2 (*)[C::ROWS][C::UBUF]>(pool + C::TAB + C::WAVES * C::ROWS * C::EXCH);
  const float2 cf = k3p_tables<N>(tab, a.window, a.scale, threadIdx.x, C::BLOCK);
  __syncthreads();

  // wave-uniform, and said so: row indices and P row pointers then live in
  // scalar registers and each store addresses P as scalar base + lane offset
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int g = lane / T;
  const int t0 = lane - g * T;
  float2* lds = xch[wave][g];
  float2* ub = ubuf[wave][g] + 1;                        // ub[i] = u[i], i in [-1, N/4+1]

  const int stride = gridDim.x * C::WAVES;
  float2 uv[4];  // the next row's taps, loaded during this one
  k3p_zero_pads<N>(ub, t0);
  {
    const int grp = blockIdx.x * C::WAVES + wave;
    if (grp < total_groups) {
      k3p_load_taps<N>(uv, a.U + (int64_t)(grp * C::ROWS + g) * a.n_cp, a.n_cp, t0);
      k3p_put_taps<N>(ub, uv, a.n_cp, t0);
    }
  }
  for (int grp = blockIdx.x * C::WAVES + wave; grp < total_groups; grp += stride) {
    const int grow = grp * C::ROWS + g;                   // row over all frames
    const int f = grow / a.m_pad;
    const int row = grow - f * a.m_pad;
    // the team lane, opaque to the optimiser, so that the per-element LDS
    // addresses are formed again for every row rather than held in registers
    // (an empty asm statement emits no instruction): what lets the one-store
    // order fit; the other forms keep the addresses, which costs them no
    // spill.  The mask restores the known range t < T, which resolves the
    // phase-0 filter's bounds tests at compile time.
    int t = t0;
    if constexpr (kOneStore) {
      asm volatile("" : "+v"(t));
      t &= T - 1;
    }
    const int gnext = grp + stride;
    const auto next = [&] {
      if (gnext < total_groups) k3p_load_taps<N>(uv, a.U + (int64_t)(gnext * C::ROWS + g) * a.n_cp, a.n_cp, t);
    };
    float mx;
    if constexpr (kStore) {
      // the job table is read-only for the whole launch: read through the
      // constant address space, a wave-uniform entry comes by a scalar load,
      // which the vector-memory waits do not count
      const auto* crefs = (const __attribute__((address_space(4))) FrameRef*)a.refs;
      const RowToGlobal sink{gptr(kRefs ? crefs[f].P : a.P + (int64_t)f * a.p_stride) + (int64_t)row * (4 * N)};
      mx = k3p_row<N, PR>(lds, ub, t, tab, cf.x, cf.y, df, sink, next);
    } else {
      mx = k3p_row<N, PR>(lds, ub, t, tab, cf.x, cf.y, df, RowToNowhere{}, next);
    }
    if (t == 0) a.rowmax[grow] = mx;
    // the next row's tap writes must follow this row's reads of ub
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    if (gnext < total_groups) k3p_put_taps<N>(ub, uv, a.n_cp, t);
  }
}

// Clears the per-frame status and peak-count words (a fill kernel rather than
// a memset, so the sequence stays safe inside captured graphs).
__global__ void k0_clear(uint32_t* status, int32_t* n_peaks, int n_frames, const FrameRef* refs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_frames) {
    uint32_t* sp = refs ? refs[i].status : (status ? status + i : nullptr);
    int32_t* np = refs ? refs[i].n_peaks : (n_peaks ? n_peaks + i : nullptr);
    if (sp) *sp = 0u;
    if (np) *np = 0;
  }
}

}  // namespace radar
