// Time-domain frame simulation (Sec. II-B.1, Eq. 1-2 and Eq. 7-10): OFDM
// symbols with a cyclic prefix, moving point targets with delay, Doppler and
// time scaling, and the receiver's prefix removal and DFT.
//
// Time is counted in samples T0 = 1/(N df); symbol l's useful part starts at
// t_l = l Ns + Ng (Ns = N + Ng).  Target p (delay rho in samples, Doppler nu
// in bins of the M-point Doppler DFT, amplitude b) has the per-sample CFO
// eps = nu N / (M Ns) and the time-scale factor B = eps / (fc/df).  Its
// delay during symbol l is d_l = rho + B t_l (the time-scale term taken at
// the symbol's start), and while 0 <= d_l <= Ng the useful window sees only
// symbol l, so
//   y_l[m] = sum_p b_p exp(+2 pi i nu_p (t_l + m)/(M Ns)) (1/N) IDFT_N(a_l exp(-2 pi i k d_l/N))[m]
//   Y_l    = DFT_N(y_l) (+ noise).
// Each team computes one symbol: one inverse FFT per target and one forward
// FFT.  The phases are reduced to [0, 1) cycles before the FP32 sincos: the
// delay's integer part exactly in integers, the Doppler base phase of each
// symbol in FP64.
#pragma once

#include "fft.hpp"
#include "k_frame.hpp"  // team_sum

namespace radar {

struct SimArgs {
  const float2* A;                // transmitted symbols, element (l,k) at l*ld + k
  int64_t ld, frame_stride;       // also the layout of noise and Y
  const radar_sim_target* targets;  // [F][max_targets]
  const int32_t* n_targets;       // [F]
  int max_targets;
  const float2* noise;            // or null
  float2* Y;
  uint32_t* status;               // [F] or null
  int M, n_guard;
  double fc_over_df;
};

template <int N>
__global__ void __launch_bounds__(kBlock) k_simulate(SimArgs a) {
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

  const float2* x = a.A + f * a.frame_stride + (int64_t)lc * a.ld;
  float2 av[16], acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    av[e] = x[t + T * e];
    acc[e] = make_float2(0.0f, 0.0f);
  }
  const double ns = (double)(N + a.n_guard);
  const double tl = (double)lc * ns + (double)a.n_guard;
  int np = a.n_targets[f];
  np = np < 0 ? 0 : (np > a.max_targets ? a.max_targets : np);
  uint32_t st = 0;
  for (int p = 0; p < np; ++p) {
    const radar_sim_target tg = a.targets[(int64_t)f * a.max_targets + p];
    const double eps = (double)tg.nu * (double)N / ((double)a.M * ns);
    const double d = (double)tg.rho + eps / a.fc_over_df * tl;  // delay during this symbol
    st |= (d >= 0.0 && d <= (double)a.n_guard) ? 0u : 4u;
    const double dfl = floor(d);
    const uint32_t dint = (uint32_t)(int64_t)dfl & (uint32_t)(N - 1);
    const float dfrac = (float)(d - dfl);
    float2 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t k = (uint32_t)(t + T * e);
      // k d / N cycles: the integer part of d exactly, then the fraction
      float cyc = (float)((k * dint) & (uint32_t)(N - 1)) * (1.0f / N) + (float)k * dfrac * (1.0f / N);
      cyc -= floorf(cyc);
      float sn, cs;
      sincospif(2.0f * cyc, &sn, &cs);
      v[e] = cmulc(av[e], make_float2(cs, sn));  // a exp(-2 pi i k d / N)
    }
    team_fft<N, 16, true>(v, lds, t);            // sum_k ... exp(+2 pi i k m / N), m = t + T e
    // Doppler: nu (t_l + m) / (M Ns) cycles, the symbol's base phase reduced in FP64
    const double base_d = (double)tg.nu * tl / ((double)a.M * ns);
    const float base = (float)(base_d - floor(base_d));
    const float inc = (float)((double)tg.nu / ((double)a.M * ns));
    const float2 bn = make_float2(tg.b_re * (1.0f / N), tg.b_im * (1.0f / N));
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      float cyc = base + (float)(t + T * e) * inc;
      cyc -= floorf(cyc);
      float sn, cs;
      sincospif(2.0f * cyc, &sn, &cs);
      acc[e] = cadd(acc[e], cmul(cmul(v[e], make_float2(cs, sn)), bn));
    }
  }
  team_fft<N, 16, false>(acc, lds, t);            // the receiver's DFT
  if (!active) return;
  const float2* z = a.noise ? a.noise + f * a.frame_stride + (int64_t)l * a.ld : nullptr;
  float2* out = a.Y + f * a.frame_stride + (int64_t)l * a.ld;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int k = t + T * e;
    out[k] = z ? cadd(acc[e], z[k]) : acc[e];
  }
  if (st && a.status) atomicOr(a.status + f, st);
}

// Peak-to-average power ratio of Eq. 25 for every OFDM symbol: the N-point
// IDFT of the symbol's subcarriers (the prefix only repeats samples), then
// max |x|^2 / mean |x|^2 over the team.  One team per symbol.
template <int N>
__global__ void __launch_bounds__(kBlock) k_papr(const float2* A, int64_t ld, int64_t frame_stride, int M,
                                                 float* papr) {
  constexpr int T = N / 16;
  constexpr int TEAMS = kBlock / T;
  __shared__ float2 lds_all[TEAMS * LdsSize<N>::value];
  __shared__ float red[2][T > 64 ? TEAMS * (T / 64) : 1];
  const int team = threadIdx.x / T;
  const int t = threadIdx.x - team * T;
  const int f = blockIdx.y;
  const int l = blockIdx.x * TEAMS + team;
  const bool active = l < M;
  const float2* x = A + f * frame_stride + (int64_t)(active ? l : 0) * ld;
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = x[t + T * e];
  team_fft<N, 16, true>(v, lds_all + team * LdsSize<N>::value, t);
  float mx = 0.0f, sum = 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const float p = cabs2(v[e]);
    mx = fmaxf(mx, p);
    sum += p;
  }
#pragma unroll
  for (int m = (T < 64 ? T : 64) / 2; m > 0; m >>= 1) {
    mx = fmaxf(mx, __shfl_xor(mx, m));
    sum += __shfl_xor(sum, m);
  }
  if constexpr (T > 64) {
    if ((t & 63) == 0) {
      red[0][team * (T / 64) + (t >> 6)] = mx;
      red[1][team * (T / 64) + (t >> 6)] = sum;
    }
    __syncthreads();
    mx = 0.0f;
    sum = 0.0f;
#pragma unroll
    for (int w = 0; w < T / 64; ++w) {
      mx = fmaxf(mx, red[0][team * (T / 64) + w]);
      sum += red[1][team * (T / 64) + w];
    }
  }
  if (active && t == 0) papr[(int64_t)f * M + l] = sum > 0.0f ? mx * (float)N / sum : 0.0f;
}

// The high power amplifier of Eq. 26 on every symbol's transmitted samples:
// x = IDFT_N(a), |x'| = |x| / sqrt(1 + (|x| / s)^2) with s = xbar 10^{q/10}
// (xbar the mean of |x| over the symbol), the phase kept, then a' = DFT_N(x').
// One team per symbol; in place allowed (out == A).
template <int N>
__global__ void __launch_bounds__(kBlock) k_hpa(const float2* A, float2* out, int64_t ld, int64_t frame_stride,
                                                int M, float sat_factor) {
  constexpr int T = N / 16;
  constexpr int TEAMS = kBlock / T;
  __shared__ float2 lds_all[TEAMS * LdsSize<N>::value];
  __shared__ float red[T > 64 ? TEAMS * (T / 64) : 1];
  const int team = threadIdx.x / T;
  const int t = threadIdx.x - team * T;
  const int f = blockIdx.y;
  const int l = blockIdx.x * TEAMS + team;
  const bool active = l < M;
  float2* lds = lds_all + team * LdsSize<N>::value;
  const int64_t off = f * frame_stride + (int64_t)(active ? l : 0) * ld;
  float2 v[16];
  float amp[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = A[off + t + T * e];
  team_fft<N, 16, true>(v, lds, t);  // N x (the samples)
  float sum = 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    v[e] = cscale(v[e], 1.0f / N);
    amp[e] = sqrtf(cabs2(v[e]));
    sum += amp[e];
  }
  sum = team_sum<T>(sum, red, team, t);
  const float sat = sum * (1.0f / N) * sat_factor;
  const float inv_sat = sat > 0.0f ? 1.0f / sat : 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const float r = amp[e] * inv_sat;
    v[e] = cscale(v[e], 1.0f / sqrtf(1.0f + r * r));
  }
  team_fft<N, 16, false>(v, lds, t);
  if (!active) return;
#pragma unroll
  for (int e = 0; e < 16; ++e) out[off + t + T * e] = v[e];
}

}  // namespace radar
