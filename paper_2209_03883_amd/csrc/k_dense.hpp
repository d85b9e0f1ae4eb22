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

#include "device_common.hpp"

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

}  // namespace radar
