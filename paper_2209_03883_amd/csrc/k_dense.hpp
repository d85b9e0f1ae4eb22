// Dense Zadoff-Chu precoding (Sec. III-B, Eq. 24 read literally with L = N^2)
// and the LS estimate of Eq. 16 against the precoded symbols.
//
// Z_m[i][j] = zc_L(iN + j) factorises, from (iN + j)^2 = i^2 N^2 + 2ijN + j^2,
// as D1 F D2 with
//   D2(j)   = exp(+i pi r (j^2 + 2qj) / N^2)
//   F(i, j) = exp(+2 pi i r ij / N)
//   D1(i)   = exp(+i pi r (N i^2 + 2qi) / N),
// so the precoded symbol a_p = Z_m a / sqrt(N) costs one N-point FFT:
//   b_j = D2(j) a_j,   X_m = sum_j b_j exp(+2 pi i mj / N),
//   a_p,i = D1(i) X_{ri mod N} / sqrt(N).
// The precoded symbols are close to complex Gaussian, so h = y / a_p is
// ill-conditioned where |a_p| is small: an FP32 transform's rounding error,
// divided by such an a_p, would dominate the noise it carries into P.  The
// transform and the division therefore run in FP64 (the vector FP64 rate
// equals the unpacked FP32 rate), and h leaves rounded once to FP32 for the
// taps stage, which then reads it as a ready LS estimate.
#pragma once

#include <utility>

#include "device_common.hpp"
#include "fft.hpp"
#include "k_frame.hpp"

// exp(+2 pi i x / 2^25) = g_root64_hi[x >> 12] * g_root64_lo[x & 4095]: FP64
// roots of unity of every power-of-two order up to 2^25 from two small tables
// (each entry rounded once on the host).
#define RADAR_ROOT64_LOG2 25
extern __device__ double2 g_root64_hi[1 << (RADAR_ROOT64_LOG2 - 12)];
extern __device__ double2 g_root64_lo[1 << 12];

namespace radar {

constexpr int kDenseThreads = 256;

// exp(+2 pi i m / 2^lg) for lg <= 25 and m < 2^lg
__device__ __forceinline__ void root64(uint32_t m, int lg, double& re, double& im) {
  const uint32_t x = m << (RADAR_ROOT64_LOG2 - lg);
  const double2 a = g_root64_hi[x >> 12], b = g_root64_lo[x & 4095u];
  re = a.x * b.x - a.y * b.y;
  im = a.x * b.y + a.y * b.x;
}

struct DenseArgs {
  const float2* Y;        // frames, element (l,k) at l*ld + k
  const float2* A;        // known (unprecoded) symbols, same layout
  int64_t ld;
  int64_t frame_stride;
  const FrameRef* refs;   // per-frame Y, A, status (batch jobs), or null
  uint32_t* status;       // [F] or null
  float2* H;              // [F][M][N] LS estimate out
  float* inv_sum;         // [F][M] sum_k 1/|a_p|^2 per symbol (threshold detection), or null
  int M;
  int total;              // F * M symbols
  uint32_t zc_root, zc_shift;  // modulo 2N^2 (2N^2 divides 2^32: uint32 products wrap exactly)
};

__device__ __forceinline__ double2 cmul64(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One Stockham stage of radix R (2 or 4) of an N-point transform with
// exp(+2 pi i ...) kernels over LDS, for sub-transforms of length ns: task j
// (j < N/R) takes d[j + r N/R], twiddles element r by exp(+2 pi i k r/(ns R))
// (k = j mod ns; tw[x] = exp(+2 pi i x/N)), runs the R-point DFT and writes
// d[(j - k) R + k + r ns].  Inputs are read into registers before the
// barrier, so the stage runs in place.
template <int N, int R>
__device__ __forceinline__ void stage64(double2* d, const double2* tw, int tid, int ns) {
  constexpr int T = kDenseThreads;
  constexpr int TASKS = N / R;
  constexpr int TPT = (TASKS + T - 1) / T;
  double2 v[TPT][R];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const int j = tid + t * T;
    if (j < TASKS) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = d[j + r * TASKS];
    }
  }
  __syncthreads();
  const int tws = N / (ns * R);
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const int j = tid + t * T;
    if (j < TASKS) {
      const int k = j & (ns - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) v[t][r] = cmul64(v[t][r], tw[k * r * tws]);
      double2 o[R];
      if constexpr (R == 2) {
        o[0] = make_double2(v[t][0].x + v[t][1].x, v[t][0].y + v[t][1].y);
        o[1] = make_double2(v[t][0].x - v[t][1].x, v[t][0].y - v[t][1].y);
      } else {
        // X_q = sum_r v_r i^{qr}
        const double2 a0 = make_double2(v[t][0].x + v[t][2].x, v[t][0].y + v[t][2].y);
        const double2 a1 = make_double2(v[t][0].x - v[t][2].x, v[t][0].y - v[t][2].y);
        const double2 a2 = make_double2(v[t][1].x + v[t][3].x, v[t][1].y + v[t][3].y);
        const double2 a3 = make_double2(-(v[t][1].y - v[t][3].y), v[t][1].x - v[t][3].x);  // i (v1 - v3)
        o[0] = make_double2(a0.x + a2.x, a0.y + a2.y);
        o[2] = make_double2(a0.x - a2.x, a0.y - a2.y);
        o[1] = make_double2(a1.x + a3.x, a1.y + a3.y);
        o[3] = make_double2(a1.x - a3.x, a1.y - a3.y);
      }
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) d[base + r * ns] = o[r];
    }
  }
  __syncthreads();
}

// X_m = sum_j d_j exp(+2 pi i mj/N) in place, natural order in and out: a
// radix-2 stage first when log2 N is odd, radix 4 after.
template <int N>
__device__ __forceinline__ void fft64(double2* d, const double2* tw, int tid) {
  int ns = 1;
  if constexpr (ilog2c(N) & 1) {
    stage64<N, 2>(d, tw, tid, ns);
    ns = 2;
  }
  for (; ns < N; ns *= 4) stage64<N, 4>(d, tw, tid, ns);
}

// One work-group per OFDM symbol at a time, persistent over the symbols of
// all frames.
template <int N>
__global__ void __launch_bounds__(kDenseThreads) k_dense_ls(DenseArgs a) {
  constexpr int T = kDenseThreads;
  constexpr int LOG = ilog2c(N);
  constexpr uint32_t kPhaseMask = 2u * (uint32_t)N * (uint32_t)N - 1u;
  __shared__ double2 s_d[N];
  __shared__ double2 s_tw[N];  // exp(+2 pi i x/N)
  __shared__ double s_red[T / 64];
  const int tid = threadIdx.x;
  for (int x = tid; x < N; x += T) root64((uint32_t)x, LOG, s_tw[x].x, s_tw[x].y);
  const double inv_sqrt_n = 1.0 / sqrt((double)N);

  for (int sym = blockIdx.x; sym < a.total; sym += gridDim.x) {
    const int f = sym / a.M;
    const int l = sym - f * a.M;
    const float2* y = (a.refs ? a.refs[f].Y : a.Y + f * a.frame_stride) + (int64_t)l * a.ld;
    const float2* x = (a.refs ? a.refs[f].A : a.A + f * a.frame_stride) + (int64_t)l * a.ld;
    // up to four elements per thread (N <= 1024), every load of the symbol is
    // issued first (a load per loop iteration with a wait before its use
    // would serialise the memory latency); longer symbols keep the loads in
    // the loops, as their transform leaves no registers to hold them
    constexpr int NT = (N + T - 1) / T;
    constexpr bool kPre = NT <= 4;
    float2 xa[kPre ? NT : 1], ya[kPre ? NT : 1];
    if constexpr (kPre) {
#pragma unroll
      for (int it = 0; it < NT; ++it) {
        const int j = tid + it * T;
        xa[it] = j < N ? x[j] : make_float2(0.0f, 0.0f);
        ya[it] = j < N ? y[j] : make_float2(0.0f, 0.0f);
      }
    }
    __syncthreads();  // the twiddles are written, the previous symbol's reads are done
#pragma unroll
    for (int it = 0; it < NT; ++it) {
      const int j = tid + it * T;
      if (j >= N) continue;  // only when N < the work-group size
      float2 av;
      if constexpr (kPre) av = xa[it];
      else av = x[j];
      const uint32_t uj = (uint32_t)j;
      const uint32_t m = (a.zc_root * (uj * uj + 2u * a.zc_shift * uj)) & kPhaseMask;
      double cs, sn;
      root64(m, 2 * LOG + 1, cs, sn);  // D2(j) = exp(+2 pi i m / 2N^2)
      s_d[j] = make_double2((double)av.x * cs - (double)av.y * sn, (double)av.x * sn + (double)av.y * cs);
    }
    __syncthreads();
    fft64<N>(s_d, s_tw, tid);
    double isum = 0.0;
    uint32_t st = 0;
    float2* h = a.H + (int64_t)sym * N;
#pragma unroll
    for (int it = 0; it < NT; ++it) {
      const int i = tid + it * T;
      if (i >= N) continue;
      const uint32_t ui = (uint32_t)i;
      const double2 xv = s_d[(a.zc_root * ui) & (uint32_t)(N - 1)];
      // D1(i) = exp(+i pi r i^2) exp(+2 pi i rqi/N) = (-1)^i W^{rqi} for odd r
      const double2 w = s_tw[(a.zc_root * a.zc_shift * ui) & (uint32_t)(N - 1)];
      const double sg = (i & 1) ? -inv_sqrt_n : inv_sqrt_n;
      const double xr = xv.x * sg, xi = xv.y * sg;
      // a_p,i, accurate in FP64, then rounded once: from here on its own
      // relative rounding (not the transform's absolute error) is what counts,
      // so the division runs in FP32
      const float2 ap = make_float2((float)(xr * w.x - xi * w.y), (float)(xr * w.y + xi * w.x));
      float2 yv;
      if constexpr (kPre) yv = ya[it];
      else yv = y[i];
      const float den = ap.x * ap.x + ap.y * ap.y;
      st |= den == 0.0f ? 1u : 0u;
      const float inv = den == 0.0f ? 0.0f : __builtin_amdgcn_rcpf(den);
      isum += (double)inv;
      // h = y conj(a_p) / |a_p|^2
      const float hr = (yv.x * ap.x + yv.y * ap.y) * inv;
      const float hi = (yv.y * ap.x - yv.x * ap.y) * inv;
      st |= (__builtin_isfinite(hr) && __builtin_isfinite(hi)) ? 0u : 2u;
      h[i] = make_float2(hr, hi);
    }
    if (a.inv_sum) {
#pragma unroll
      for (int m = 32; m > 0; m >>= 1) isum += __shfl_xor(isum, m);
      if ((tid & 63) == 0) s_red[tid >> 6] = isum;
      __syncthreads();
      if (tid == 0) {
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < T / 64; ++w) tot += s_red[w];
        a.inv_sum[sym] = (float)tot;
      }
    }
    if (st) {
      uint32_t* sp = a.refs ? a.refs[f].status : (a.status ? a.status + f : nullptr);
      if (sp) atomicOr(sp, st);
    }
  }
}

// ------------------------------------------------------------------------
// The dense precoding fused into the taps stage (N = 256 .. 1024): one team
// of T = N/16 lanes per OFDM symbol, as in k1_taps_p, with the precoded
// symbols' FP64 transform done by the team itself:
//   b_j = D2(j) a_j,  X = sum_j b_j exp(+2 pi i mj/N)  (FP64, in registers),
//   a_p,i = D1(i) X_{ri mod N} / sqrt(N)  (FP64, rounded once to FP32),
//   h_i = y_i conj(a_p,i) / |a_p,i|^2,  taps = w_l/N IDFT_N(h), n < N_cp (FP32).
// The FP64 transform is a Stockham FFT of the same shape as the FP32 one in
// fft.hpp (16 values per lane in the cyclic layout v[e] = x[t + T e], radix
// 16 stages, a smaller last radix) whose exchanges pass real and imaginary
// parts in turn through the team's FP32 exchange region (N + N/16 8-byte
// entries), so the team syncs at wave scope only.  The LS estimate never
// leaves the chip.
// ------------------------------------------------------------------------

// a exp(+2 pi i Q/16) in FP64
template <int Q>
__device__ __forceinline__ double2 rot16p64(double2 a) {
  constexpr int q = Q & 15;
  constexpr double kc[16] = {1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
                             0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
                             -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977,
                             0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674};
  constexpr double ks[16] = {0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674,
                             1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
                             0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
                             -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977};
  if constexpr (q == 0) {
    return a;
  } else if constexpr (q == 4) {
    return make_double2(-a.y, a.x);
  } else if constexpr (q == 8) {
    return make_double2(-a.x, -a.y);
  } else if constexpr (q == 12) {
    return make_double2(a.y, -a.x);
  } else {
    return make_double2(a.x * kc[q] - a.y * ks[q], a.y * kc[q] + a.x * ks[q]);
  }
}

// R-point DFT with exp(+2 pi i qr/R) kernel, in place, by radix-2
// decimation in time (R = 2, 4, 8, 16).
template <int R>
struct Dft64 {
  template <int K>
  static __device__ __forceinline__ void combine(double2* x, const double2* e, const double2* o) {
    const double2 t = rot16p64<K * (16 / R)>(o[K]);
    x[K] = make_double2(e[K].x + t.x, e[K].y + t.y);
    x[K + R / 2] = make_double2(e[K].x - t.x, e[K].y - t.y);
  }
  template <int... K>
  static __device__ __forceinline__ void combine_all(double2* x, const double2* e, const double2* o,
                                                     std::integer_sequence<int, K...>) {
    (combine<K>(x, e, o), ...);
  }
  static __device__ __forceinline__ void run(double2* x) {
    double2 e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    Dft64<R / 2>::run(e);
    Dft64<R / 2>::run(o);
    combine_all(x, e, o, std::make_integer_sequence<int, R / 2>{});
  }
};
template <>
struct Dft64<1> {
  static __device__ __forceinline__ void run(double2*) {}
};

// One exchange of the team's 16 values through the FP32-sized region: the
// value for position pos[e] is written, then element e of the cyclic layout
// read back, real parts first, then imaginary parts.
template <int T, class PosF>
__device__ __forceinline__ void xch64(double2 (&v)[16], double* dl, int t, const PosF& pos) {
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
    for (int e = 0; e < 16; ++e) dl[lds_pad(pos(e))] = pass ? v[e].y : v[e].x;
    team_sync<T>();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const double r = dl[lds_pad(t + T * e)];
      if (pass) v[e].y = r;
      else v[e].x = r;
    }
    // this pass's reads come before the next pass's writes (in order on the LDS)
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// Stages from span NS on of the N-point transform (exp(+) kernel) of the
// team's values (T = N/16 lanes, lane t); tw[x] = exp(+2 pi i x/N).
template <int N, int NS>
__device__ __forceinline__ void fft64_stages(double2 (&v)[16], double* dl, int t, const double2* tw) {
  constexpr int T = N / 16;
  constexpr int REM = N / NS;
  constexpr int R = REM >= 16 ? 16 : REM;
  constexpr int NB = 16 / R;
  constexpr bool LAST = NS * R == N;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double2 x[R];
#pragma unroll
    for (int m = 0; m < R; ++m) x[m] = v[b + m * NB];
    const int j = t + T * b;
    const int k = j & (NS - 1);
    if constexpr (NS > 1) {
#pragma unroll
      for (int m = 1; m < R; ++m) x[m] = cmul64(x[m], tw[(k * m * (N / (NS * R))) & (N - 1)]);
    }
    Dft64<R>::run(x);
#pragma unroll
    for (int m = 0; m < R; ++m) v[b + m * NB] = x[m];
  }
  if constexpr (!LAST) {
    // output m of butterfly j (element b + m NB) goes to (j - k) R + k + m NS
    xch64<T>(v, dl, t, [&](int e) {
      const int b = e % NB, m = e / NB;
      const int j = t + T * b;
      const int k = j & (NS - 1);
      return (j - k) * R + k + m * NS;
    });
    fft64_stages<N, NS * R>(v, dl, t, tw);
  }
}

template <int N>
struct K1d {
  static constexpr int T = N / 16;
  static constexpr int ROWS = 64 / T;                     // symbols per wave per pass
  static constexpr int WAVES = 8;
  static constexpr int BLOCK = 64 * WAVES;
  static constexpr int TAB = PlanTable<N, 16, 1>::size();  // the FP32 inverse plan's stage blocks
  static constexpr int EXCH = LdsSize<N>::value;
  using Inv = PlanLayout<N, 0, 1>;
};

template <int N>
__global__ void __launch_bounds__(K1d<N>::BLOCK) k1_taps_dense(K1Args a, int total_groups) {
  using C = K1d<N>;
  constexpr int T = C::T;
  constexpr int LOG = ilog2c(N);
  constexpr uint32_t kPhaseMask = 2u * (uint32_t)N * (uint32_t)N - 1u;
  __shared__ float2 tab[C::TAB > 0 ? C::TAB : 1];
  __shared__ double2 tw64[N];  // exp(+2 pi i x/N)
  __shared__ double2 d2[N];    // D2(j): the launch's root and shift fix it for every symbol
  __shared__ float2 xch[C::WAVES][C::ROWS][C::EXCH];
  copy_plan_twiddles<N, 16, 1>(tab, threadIdx.x, C::BLOCK);
  for (int x = threadIdx.x; x < N; x += C::BLOCK) {
    root64((uint32_t)x, LOG, tw64[x].x, tw64[x].y);
    const uint32_t uj = (uint32_t)x;
    const uint32_t m = (a.zc_root * (uj * uj + 2u * a.zc_shift * uj)) & kPhaseMask;
    root64(m, 2 * LOG + 1, d2[x].x, d2[x].y);  // exp(+2 pi i m / 2N^2)
  }
  __syncthreads();
  const TwLds<typename C::Inv> tw_inv{tab};
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane / T;
  const int t0 = lane - g * T;
  float2* lds = xch[wave][g];
  double* dl = reinterpret_cast<double*>(lds);
  const double inv_sqrt_n = 1.0 / sqrt((double)N);

  for (int grp = blockIdx.x * C::WAVES + wave; grp < total_groups; grp += gridDim.x * C::WAVES) {
    // the lane, opaque to the optimiser: per-element addresses are formed
    // again per symbol rather than held in registers
    int t = t0;
    asm volatile("" : "+v"(t));
    t &= T - 1;
    const int gsym = grp * C::ROWS + g;  // symbol over all frames
    const int f = gsym / a.M;
    const int l = gsym - f * a.M;
    const RADAR_GLOBAL float2* y = gptr(a.refs ? a.refs[f].Y : a.Y + f * a.frame_stride) + l * a.ld;
    const RADAR_GLOBAL float2* x = gptr(a.refs ? a.refs[f].A : a.A + f * a.frame_stride) + l * a.ld;
    double2 v[16];
    float2 yv[16];  // the received symbol, loaded now, used after the transform
    {
      float2 av[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) av[e] = gload2(x + t + T * e);
#pragma unroll
      for (int e = 0; e < 16; ++e) yv[e] = gload2(y + t + T * e);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const double2 w = d2[t + T * e];  // b_j = D2(j) a_j
        v[e] = make_double2((double)av[e].x * w.x - (double)av[e].y * w.y, (double)av[e].x * w.y + (double)av[e].y * w.x);
      }
    }
    fft64_stages<N, 1>(v, dl, t, tw64);  // X_m, m = t + T e
    // a_p,i needs X at r i mod N: through the exchange region, real and
    // imaginary parts in turn
    asm volatile("" : "+v"(t));
    t &= T - 1;
    double2 xp[16];
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
      for (int e = 0; e < 16; ++e) dl[lds_pad(t + T * e)] = pass ? v[e].y : v[e].x;
      team_sync<T>();
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const uint32_t i = (uint32_t)(t + T * e);
        const double r = dl[lds_pad((int)((a.zc_root * i) & (uint32_t)(N - 1)))];
        if (pass) xp[e].y = r;
        else xp[e].x = r;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    uint32_t st = 0;
    float isum = 0.0f;
    float2 hv[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t i = (uint32_t)(t + T * e);
      // D1(i) = (-1)^i exp(+2 pi i rqi/N) for odd r
      const double2 w = tw64[(a.zc_root * a.zc_shift * i) & (uint32_t)(N - 1)];
      const double sg = (i & 1u) ? -inv_sqrt_n : inv_sqrt_n;
      const double xr = xp[e].x * sg, xi = xp[e].y * sg;
      // a_p,i accurate in FP64, then rounded once; the division runs in FP32
      const float2 ap = make_float2((float)(xr * w.x - xi * w.y), (float)(xr * w.y + xi * w.x));
      const float den = ap.x * ap.x + ap.y * ap.y;
      st |= den == 0.0f ? 1u : 0u;
      const float inv = den == 0.0f ? 0.0f : __builtin_amdgcn_rcpf(den);
      isum += inv;
      hv[e] = make_float2((yv[e].x * ap.x + yv[e].y * ap.y) * inv, (yv[e].y * ap.x - yv[e].x * ap.y) * inv);
      st |= (__builtin_isfinite(hv[e].x) && __builtin_isfinite(hv[e].y)) ? 0u : 2u;
    }
    if (a.inv_sum) {
      isum = team_sum<T>(isum, nullptr, 0, t);
      if (t == 0) a.inv_sum[gsym] = isum;
    }
    fft_stages<N, 16, 1, true>(hv, lds, t, true, tw_inv);
    const float scale = window_value(a.window, l, a.M) * a.inv_n;
    float2* out = a.taps + (int64_t)gsym * a.n_cp;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int n = t + T * e;
      if (n < a.n_cp) out[n] = cscale(hv[e], a.tap_w ? scale * a.tap_w[n] : scale);
    }
    if (st) {
      uint32_t* sp = a.refs ? a.refs[f].status : (a.status ? a.status + f : nullptr);
      if (sp) atomicOr(sp, st);
    }
  }
}

}  // namespace radar
