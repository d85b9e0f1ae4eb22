// Sub-cell refinement of detected peaks (K7).
//
// For a peak at padded cell (s, r) the periodogram padded 16x in both axes is
// evaluated on the 7 x 7 fine cells around it, straight from the DFT-CE taps
// t_l[n] (which already carry w_l and 1/N):
//   V_a[n]  = sum_l t_l[n] e^{-2 pi i l sigma_a / M}            sigma_a = (cs + a - 3)/16  (FP32)
//   G_ab    = sum_n V_a[n] K(rho_b - n),  rho_b = (cr + b - 3)/16                        (FP64)
//   K(x)    = sum_{k<N} w_k e^{+2 pi i k x / N} = a0 D(x) - a1/2 (D(x+1) + D(x-1)),
//   D(x)    = sum_{k<N} e^{2 pi i k x/N} = e^{i pi x (N-1)/N} sin(pi x)/sin(pi x/N)
//   P_ab    = |G_ab|^2 / (N M)
// (cs, cr: the peak's fine indices).  The best fine cell of the inner 5 x 5
// and a least-squares quadratic of ln P over its 3 x 3 neighbourhood, solved in
// FP64, give the sub-cell position (separable parabolas when the quadratic has
// no maximum within one cell).
#pragma once

#include "device_common.hpp"
#include "../../include/radar.h"

namespace radar {

struct K7Args {
  const float2* taps;      // [F][M][n_cp]
  radar_peak* peaks;       // [F][k]
  const int32_t* n_peaks;  // [F]
  int k, M, N, n_cp, m_pad, n_pad, window;
  const FrameRef* refs;    // per-frame peaks / n_peaks (batch jobs), or null
};

constexpr int kRefineThreads = 1024;
constexpr int kRefineNChunk = 256;                         // taps per pass
constexpr int kRefineLSplit = kRefineThreads / kRefineNChunk;  // symbol ranges summed in parallel

__device__ __forceinline__ double2 dirichlet(double x, int N) {
  // sum_{k<N} e^{2 pi i k x/N}; x = q/16 with q an integer, so x/N = 0 mod 1 only
  // when every term is 1
  const double den = sinpi(x / N);
  if (fabs(den) < 1e-300) return make_double2((double)N, 0.0);
  const double mag = sinpi(x) / den;
  const double ph = x * (double)(N - 1) / (double)N;
  return make_double2(mag * cospi(ph), mag * sinpi(ph));
}

__global__ void __launch_bounds__(kRefineThreads) k7_refine(K7Args a) {
  __shared__ float2 s_part[kRefineLSplit][7][kRefineNChunk];  // partial Doppler sums
  __shared__ double2 s_v[7][kRefineNChunk];
  __shared__ double2 s_D[7][kRefineNChunk + 2];  // D(rho_y - n) for n = n0 - 1 .. n0 + chunk
  __shared__ double2 s_g[7][7];  // holds P[7][7] (as doubles) for the fit
  __shared__ double2 s_red[16][7 * 7];
  const int f = blockIdx.y;
  const int i = blockIdx.x;
  if (i >= (a.refs ? *a.refs[f].n_peaks : a.n_peaks[f])) return;
  radar_peak* pk = (a.refs ? a.refs[f].peaks : a.peaks + (int64_t)f * a.k) + i;
  const int fs = 16 * a.M / a.m_pad;   // fine cells per padded cell
  const int fr = 16 * a.N / a.n_pad;
  const int cs = pk->s * fs;           // signed fine Doppler index
  const int cr = pk->r * fr;           // fine range index
  const int tid = threadIdx.x;
  const int nl = tid % kRefineNChunk;
  const int q = tid / kRefineNChunk;
  const int lchunk = (a.M + kRefineLSplit - 1) / kRefineLSplit;
  const int l0 = q * lchunk, l1 = min(a.M, l0 + lchunk);
  const int L16 = 16 * a.M;            // Doppler twiddles W_{16M}^x (16M <= LMAX)
  const float2* tp = a.taps + (int64_t)f * a.M * a.n_cp;

  double2 gacc = make_double2(0.0, 0.0);  // thread tid < 49 owns fine cell (tid / 7, tid % 7)

  const float2 wc = window_coeffs(a.window);
  for (int n0 = 0; n0 < a.n_cp; n0 += kRefineNChunk) {
    const int n = n0 + nl;
    float2 acc[7];
#pragma unroll
    for (int x = 0; x < 7; ++x) acc[x] = make_float2(0.0f, 0.0f);
    if (n < a.n_cp) {
      for (int l = l0; l < l1; ++l) {
        const float2 t = tp[(int64_t)l * a.n_cp + n];
#pragma unroll
        for (int x = 0; x < 7; ++x) {
          const int e = (l * (cs + x - 3)) & (L16 - 1);  // mod 16M (a power of two)
          const float2 w = twiddle(L16, e);               // e^{-2 pi i l sigma/M}
          acc[x] = cadd(acc[x], cmul(t, w));
        }
      }
    }
#pragma unroll
    for (int x = 0; x < 7; ++x) s_part[q][x][nl] = acc[x];
    __syncthreads();
    if (tid < kRefineNChunk) {
#pragma unroll
      for (int x = 0; x < 7; ++x) {
        float2 v = s_part[0][x][tid];
        for (int qq = 1; qq < kRefineLSplit; ++qq) v = cadd(v, s_part[qq][x][tid]);
        s_v[x][tid] = make_double2((double)v.x, (double)v.y);
      }
    }
    // the Dirichlet kernel at every (fine range position, tap) pair of the chunk
    for (int i = tid; i < 7 * (kRefineNChunk + 2); i += kRefineThreads) {
      const int y = i / (kRefineNChunk + 2), j = i - y * (kRefineNChunk + 2);
      s_D[y][j] = dirichlet((double)(cr + y - 3 - 16 * (n0 - 1 + j)) / 16.0, a.N);
    }
    __syncthreads();
    // range sums: thread (x, y, n-slice) accumulates sum_n V_x[n] K(rho_y - n)
    if (tid < 7 * 7 * 16) {
      const int xy = tid % 49, slice = tid / 49;
      const int x = xy / 7, y = xy % 7;
      double2 g = make_double2(0.0, 0.0);
      for (int nn = slice; nn < kRefineNChunk && n0 + nn < a.n_cp; nn += 16) {
        const double2 d0 = s_D[y][nn + 1];  // D(rho_y - n)
        const double2 dp = s_D[y][nn];      // D(rho_y - n + 1)
        const double2 dm = s_D[y][nn + 2];  // D(rho_y - n - 1)
        const double kr = (double)wc.x * d0.x - 0.5 * (double)wc.y * (dp.x + dm.x);
        const double ki = (double)wc.x * d0.y - 0.5 * (double)wc.y * (dp.y + dm.y);
        const double2 v = s_v[x][nn];
        g.x += v.x * kr - v.y * ki;
        g.y += v.x * ki + v.y * kr;
      }
      s_red[slice][xy] = g;
    }
    __syncthreads();
    if (tid < 49) {
      double2 g = s_red[0][tid];
      for (int sl = 1; sl < 16; ++sl) {
        g.x += s_red[sl][tid].x;
        g.y += s_red[sl][tid].y;
      }
      gacc.x += g.x;
      gacc.y += g.y;
    }
    __syncthreads();
  }
  const double norm = 1.0 / ((double)a.N * (double)a.M);
  double(*P)[7] = reinterpret_cast<double(*)[7]>(&s_g[0][0]);  // P reuses the G cells' storage
  if (tid < 49) P[tid / 7][tid % 7] = (gacc.x * gacc.x + gacc.y * gacc.y) * norm;
  __syncthreads();
  if (tid != 0) return;

  // FP64 fit
  int bx = 1, by = 1;
  for (int x = 1; x < 6; ++x)
    for (int y = 1; y < 6; ++y)
      if (P[x][y] > P[bx][by]) {
        bx = x;
        by = y;
      }
  double F[3][3];
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y) F[x][y] = log(fmax(P[bx + x - 1][by + y - 1], 2.2250738585072014e-308));
  double b = 0, c = 0, e = 0, d = 0, g = 0;
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      const double xv = x - 1.0, yv = y - 1.0;
      b += xv * F[x][y];
      c += yv * F[x][y];
      e += xv * yv * F[x][y];
      d += (xv * xv - 2.0 / 3.0) * F[x][y];
      g += (yv * yv - 2.0 / 3.0) * F[x][y];
    }
  b /= 6.0;
  c /= 6.0;
  e /= 4.0;
  d /= 2.0;
  g /= 2.0;
  const double det = 4.0 * d * g - e * e;
  double ox = 0.0, oy = 0.0;
  bool done = false;
  if (d < 0 && det > 0) {
    ox = -(2.0 * g * b - e * c) / det;
    oy = -(2.0 * d * c - e * b) / det;
    done = fabs(ox) <= 1.0 && fabs(oy) <= 1.0;
  }
  if (!done) {
    const double dx = F[0][1] - 2.0 * F[1][1] + F[2][1];
    const double dy = F[1][0] - 2.0 * F[1][1] + F[1][2];
    ox = dx < 0 ? 0.5 * (F[0][1] - F[2][1]) / dx : 0.0;
    oy = dy < 0 ? 0.5 * (F[1][0] - F[1][2]) / dy : 0.0;
  }
  ox = fmin(0.5, fmax(-0.5, ox));
  oy = fmin(0.5, fmax(-0.5, oy));
  pk->s_off = (float)(((bx - 3) + ox) / fs);
  pk->r_off = (float)(((by - 3) + oy) / fr);
}

}  // namespace radar
