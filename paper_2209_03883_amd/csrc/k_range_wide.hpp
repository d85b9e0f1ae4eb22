// The range stage for N = 2048 (4x range padding, N_cp <= N/4), FP32:
// persistent work-groups, two waves per Doppler row, every length-N
// transform computed as two length-H = N/2 transforms, so that a lane holds
// 16 values of each and the length-1024 plans and LDS tables of the N <= 1024
// kernel serve unchanged.
//
// forward   X = DFT_N(u), u zero beyond N/4, split by tap parity (decimation
//           in time): with E_j = DFT_H(u[2m + j]),
//               X[k] = E_0[k] + W_N^k E_1[k],  X[k + H] = E_0[k] - W_N^k E_1[k];
//           each E_j has N/8 = H/4 nonzero inputs, so it starts at span 4
//           like the N = 1024 forward.  Wave j of the pair computes E_j and
//           the two trade them through LDS.  The window and sqrt(1/(N M))
//           then scale X (w_{k+H} = a0 + a1 cos(2 pi k/N)).
// phases    b = 1, 2, 3: g = IDFT_N(y), y[k] = X[k] W_{4N}^{-k b}.  Split by
//           output parity (decimation in frequency): for r = 2s + h,
//               g[2s + h] = IDFT_H(v_h)[s],
//               v_h[k] = W_N^{-k h} (y[k] + (-1)^h y[k + H]),
//           and y[k + H] = X[k + H] W_{4N}^{-k b} e^{+i pi b/4}, so
//               v_h[k] = W_{4N}^{-k b} W_N^{-k h} (X[k] + (-1)^h e^{i pi b/4} X[k + H]).
//           Wave h of the pair computes half h.  Row cell 4 r + b holds
//           |g[r]|^2 (Sec. IV-A: padding the range IDFT by four interleaves
//           four phase-shifted N-point IDFTs).
// phase 0   the three-tap filter of the taps, as for N <= 1024.
// stores    a wave holds the four phases of its 16 cells per lane, so each
//           four-phase group leaves in one 16-byte store.  The two waves of a
//           row run in step and write alternate groups of every line at
//           nearly the same time.  (One wave doing both
//           halves in turn left half-written lines in the caches for a third
//           of a row's time, long enough to be evicted as partial lines:
//           measured 1.7x slower; non-temporal stores, which skip that
//           joining, as slow.)
// LDS       per work-group: the two length-H plans' stage blocks, W_{4N}^{k b}
//           (b = 1..3) and W_N^k for k < H (51 KB); per wave an exchange
//           region and the row's taps.
#pragma once

#include "fft.hpp"
#include "k_frame.hpp"

namespace radar {

template <int N>
struct K3w {
  static constexpr int H = N / 2;                        // half length
  static constexpr int T = 64;                           // lanes per row (one wave)
  static constexpr int E = H / T;                        // values per lane per half
  static constexpr int WAVES = 8;
  static constexpr int PAIRS = WAVES / 2;                // rows in flight per work-group
  static constexpr int BLOCK = 64 * WAVES;
  static constexpr int FWD = 0;                          // forward plan (length H, from span 4)
  static constexpr int INV = PlanTable<H, 16, 4>::size();  // inverse plan (length H, from span 1)
  static constexpr int PH = INV + PlanTable<H, 16, 1>::size();  // W_{4N}^{k b}, b = 1..3, k < H
  static constexpr int WN = PH + 3 * H;                  // W_N^k, k < H
  static constexpr int TAB = WN + H;
  static constexpr int EXCH = LdsSize<H>::value;
  static constexpr int UBUF = N / 4 + 3;                 // u[-1 .. N/4+1]
  static constexpr int TAPS = N / 4 / T;                 // taps loaded per lane
  using Fwd = PlanLayout<H, FWD, 4>;
  using Inv = PlanLayout<H, INV, 1>;
  static_assert(E == 16, "the length-H transforms use the 16-per-lane plans");
};

// The tables (plain copies of the library twiddle table).  Returns
// (a0 rs, a1 rs) of the window, rs = sqrt(scale).
template <int N>
__device__ __forceinline__ float2 k3w_tables(float2* tab, int window, float scale, int tid, int nthreads) {
  using C = K3w<N>;
  constexpr int H = C::H;
  copy_plan_twiddles<H, 16, 4>(tab + C::FWD, tid, nthreads);
  copy_plan_twiddles<H, 16, 1>(tab + C::INV, tid, nthreads);
  constexpr int poff = phase_offset(ilog2c(N), 2);
  for (int i = tid; i < 3 * H; i += nthreads) {
    const int b = 1 + i / H, k = i - (b - 1) * H;
    tab[C::PH + i] = g_radar_tw[(unsigned)(poff + b * N + k)];  // W_{4N}^{k b}
  }
  for (int k = tid; k < H; k += nthreads) tab[C::WN + k] = g_radar_tw[(unsigned)(N + k)];  // W_N^k
  const float2 wc = window_coeffs(window);
  const float rs = sqrtf(scale);
  return make_float2(wc.x * rs, wc.y * rs);
}

template <int N>
__device__ __forceinline__ void k3w_load_taps(float2 (&uv)[K3w<N>::TAPS], const float2* in, int n_cp, int t) {
#pragma unroll
  for (int e = 0; e < K3w<N>::TAPS; ++e) {
    const int n = t + 64 * e;
    uv[e] = in[n < n_cp ? n : 0];
  }
}
template <int N>
__device__ __forceinline__ void k3w_put_taps(float2* ub, const float2 (&uv)[K3w<N>::TAPS], int n_cp, int t) {
#pragma unroll
  for (int e = 0; e < K3w<N>::TAPS; ++e) {
    const int n = t + 64 * e;
    ub[n] = n < n_cp ? uv[e] : make_float2(0.0f, 0.0f);
  }
}

// z e^{i pi b/4}, b = 1, 2, 3
template <int B>
__device__ __forceinline__ float2 rot_eighth(float2 z) {
  constexpr float s = 0.70710678118654752f;
  if constexpr (B == 1) return make_float2((z.x - z.y) * s, (z.x + z.y) * s);
  if constexpr (B == 2) return make_float2(-z.y, z.x);
  return make_float2(-(z.x + z.y) * s, (z.x - z.y) * s);
}

// The lane index, opaque to the optimiser (an empty asm statement emits no
// instruction) and masked back to its range: values derived from it are
// formed again where used rather than held in registers.
__device__ __forceinline__ int k3w_lane(int t) {
  asm volatile("" : "+v"(t));
  return t & 63;
}

// The input of half h, phase b (v_h of the header comment, for the lane's
// 16 elements) and its length-H inverse transform, left in gv.  The lane
// index is made opaque first, so that the per-element LDS addresses are
// formed afresh for each transform rather than held in registers.
template <int N, int Hf, int B, class TS>
__device__ __forceinline__ void k3w_phase(float2 (&gv)[K3w<N>::E], const float2 (&xl)[K3w<N>::E],
                                          const float2 (&xh)[K3w<N>::E], float2* lds, const float2* tab, int t,
                                          const TS& tw_inv) {
  using C = K3w<N>;
  t = k3w_lane(t);
#pragma unroll
  for (int e = 0; e < C::E; ++e) {
    const int k = t + 64 * e;
    // opaque copy: keeps the sums and differences that the rotations of
    // different phases share from being held from one phase to the next
    float2 x = xh[e];
    asm volatile("" : "+v"(x.x), "+v"(x.y));
    const float2 r = rot_eighth<B>(x);
    float2 z = Hf == 0 ? cadd(xl[e], r) : csub(xl[e], r);
    z = cmulc(z, tab[C::PH + (B - 1) * C::H + k]);
    if constexpr (Hf == 1) z = cmulc(z, tab[C::WN + k]);
    gv[e] = z;
  }
  fft_stages<C::H, C::E, 1, true>(gv, lds, t, true, tw_inv, DftFp32{});
}

// Forward half of wave parity j: E_j = DFT_H(u[2m + j]) from span 4 (element
// t + 64 e takes u[2 ((t + 64 e) / 4) + j] = u[2 (t/4 + 16 e) + j]), left in
// x in the cyclic layout.
template <int N>
__device__ __forceinline__ void k3w_forward(float2 (&x)[K3w<N>::E], float2* lds, const float2* ub, int t, int j,
                                            const float2* tab) {
  using C = K3w<N>;
#pragma unroll
  for (int e = 0; e < C::E; ++e) x[e] = ub[2 * ((t >> 2) + 16 * e) + j];
  fft_stages<C::H, C::E, 4, false>(x, lds, t, true, TwLdsLate<typename C::Fwd>{{tab}}, DftFp32{});
}

// X[k] = E_0[k] + W_N^k E_1[k] and X[k + H] = E_0[k] - W_N^k E_1[k], each
// times the window and rs (wr = (a0 rs, a1 rs)); on entry xl = E_0, xh = E_1.
template <int N>
__device__ __forceinline__ void k3w_combine(float2 (&xl)[K3w<N>::E], float2 (&xh)[K3w<N>::E], const float2* tab,
                                            int t, float2 wr) {
  using C = K3w<N>;
#pragma unroll
  for (int e = 0; e < C::E; ++e) {
    const float2 w = tab[C::WN + t + 64 * e];
    const float2 o = cmul(xh[e], w);
    const float wl = wr.x - wr.y * w.x, wh = wr.x + wr.y * w.x;  // window at k and k + H
    xh[e] = cscale(csub(xl[e], o), wh);
    xl[e] = cscale(cadd(xl[e], o), wl);
  }
}

// Half Hf of one row (the cells 4 r + b, r = 2 s + Hf): |g|^2 of phases 1,
// 2 and 3 for the lane's 16 values of s, left in p1, p2, p3.
template <int N, int Hf>
__device__ __forceinline__ void k3w_half(const float2 (&xl)[K3w<N>::E], const float2 (&xh)[K3w<N>::E], float2* lds,
                                         const float2* tab, int t, float (&p1)[K3w<N>::E], float (&p2)[K3w<N>::E],
                                         float (&p3)[K3w<N>::E]) {
  using C = K3w<N>;
  constexpr int E = C::E;
  const TwLdsLate<typename C::Inv> tw_inv{{tab}};
  {
    float2 gv[E];
    k3w_phase<N, Hf, 1>(gv, xl, xh, lds, tab, t, tw_inv);
#pragma unroll
    for (int e = 0; e < E; ++e) p1[e] = cabs2(gv[e]);
  }
  {
    float2 gv[E];
    k3w_phase<N, Hf, 2>(gv, xl, xh, lds, tab, t, tw_inv);
#pragma unroll
    for (int e = 0; e < E; ++e) p2[e] = cabs2(gv[e]);
  }
  {
    float2 gv[E];
    k3w_phase<N, Hf, 3>(gv, xl, xh, lds, tab, t, tw_inv);
#pragma unroll
    for (int e = 0; e < E; ++e) p3[e] = cabs2(gv[e]);
  }
}

// kRefs: P row pointers from the batch job table.  The work-group's waves
// run in step (every loop trip holds the same barriers for all of them; a
// pair past the last row idles through them).
template <int N, bool kRefs = false>
__global__ void __launch_bounds__(K3w<N>::BLOCK) k3_range_power_x4w(K3Args a, int total_rows) {
  using C = K3w<N>;
  constexpr int E = C::E;
  static_assert(C::TAB * 8 < 65536, "twiddle table beyond the LDS offset range");
  __shared__ float2 pool[C::TAB + C::WAVES * (C::EXCH + C::UBUF)];
  __shared__ float s_max[C::PAIRS];
  float2* const tab = pool;
  const float2 wr = k3w_tables<N>(tab, a.window, a.scale, threadIdx.x, C::BLOCK);
  const float c0 = (float)N * wr.x, c1 = -0.5f * (float)N * wr.y;
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int pair = wave >> 1, hf = wave & 1;
  const int t0 = threadIdx.x & 63;
  float2* lds = pool + C::TAB + wave * C::EXCH;
  const float2* lds_e0 = pool + C::TAB + (wave & ~1) * C::EXCH;  // the pair's E_0
  const float2* lds_e1 = lds_e0 + C::EXCH;                         // and E_1
  float2* ub = pool + C::TAB + C::WAVES * C::EXCH + wave * C::UBUF + 1;  // ub[i] = u[i], i in [-1, N/4+1]

  const int stride = gridDim.x * C::PAIRS;
  float2 uv[C::TAPS];
  k3p_zero_pads<N>(ub, t0);
  {
    const int row0 = blockIdx.x * C::PAIRS + pair;
    if (row0 < total_rows) {
      k3w_load_taps<N>(uv, a.U + (int64_t)row0 * a.n_cp, a.n_cp, t0);
      k3w_put_taps<N>(ub, uv, a.n_cp, t0);
    }
  }
  float mx_prev = 0.0f;  // this wave's maximum of its last row (row_prev)
  int row_prev = -1;
  for (int base = blockIdx.x * C::PAIRS; base < total_rows; base += stride) {
    const int grow = base + pair;
    const bool active = grow < total_rows;  // wave-uniform
    const int f = grow / a.m_pad;
    const int row = grow - f * a.m_pad;
    int t = k3w_lane(t0);
    if (active) {
      team_sync<64>();  // this wave's tap writes before its reads
      float2 own[E];
      k3w_forward<N>(own, lds, ub, t, hf, tab);
      // the transform's last exchange reads come before these writes
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
      for (int e = 0; e < E; ++e) lds[t + 64 * e] = own[e];
    }
    __syncthreads();
    // the previous row's maximum (wave 1 wrote its half's before this barrier
    // and writes again only after the next one)
    if (hf == 0 && t0 == 0 && row_prev >= 0) a.rowmax[row_prev] = fmaxf(mx_prev, s_max[pair]);
    float2 xl[E], xh[E];  // E_0 and E_1, both read back from the pair's regions
    if (active) {
      t = k3w_lane(t);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        xl[e] = lds_e0[t + 64 * e];
        xh[e] = lds_e1[t + 64 * e];
      }
    }
    __syncthreads();  // both regions are free for the transforms
    float p0[E], p1[E], p2[E], p3[E];
    if (active) {
      k3w_combine<N>(xl, xh, tab, t, wr);
      if (hf == 0)
        k3w_half<N, 0>(xl, xh, lds, tab, t, p1, p2, p3);
      else
        k3w_half<N, 1>(xl, xh, lds, tab, t, p1, p2, p3);
      // the next row's taps, loaded while this row is stored
      const int gnext = grow + stride < total_rows ? grow + stride : grow;
      k3w_load_taps<N>(uv, a.U + (int64_t)gnext * a.n_cp, a.n_cp, t);
      t = k3w_lane(t);
      float mx = 0.0f;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        p0[e] = cabs2(phase0_filter<N>(ub, 2 * (t + 64 * e) + hf, c0, c1));
        mx = fmaxf(fmaxf(fmaxf(fmaxf(mx, p0[e]), p1[e]), p2[e]), p3[e]);
      }
#pragma unroll
      for (int m = 32; m > 0; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
      // the row maximum: wave 1 leaves its half's in LDS, wave 0 combines
      // it with its own after the next trip's first barrier
      if (hf == 1 && t0 == 0) s_max[pair] = mx;
      mx_prev = mx;
      row_prev = grow;
      const auto* crefs = (const __attribute__((address_space(4))) FrameRef*)a.refs;
      RADAR_GLOBAL float* dst = gptr(kRefs ? crefs[f].P : a.P + (int64_t)f * a.p_stride) + (int64_t)row * (4 * N);
      t = k3w_lane(t);
#pragma unroll
      for (int e = 0; e < E; ++e) gstore4(dst + 4 * (2 * (t + 64 * e) + hf), p0[e], p1[e], p2[e], p3[e]);
      // the next row's tap writes follow this row's reads of ub
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      k3w_put_taps<N>(ub, uv, a.n_cp, t0);
    }
  }
  __syncthreads();
  if (hf == 0 && t0 == 0 && row_prev >= 0) a.rowmax[row_prev] = fmaxf(mx_prev, s_max[pair]);
}

}  // namespace radar
