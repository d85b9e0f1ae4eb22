// The range stage of the 4x-padded periodogram (Eq. 17, with the DFT back to
// the subcarriers of Eq. 22) on the matrix cores, for N = 1024, N' = 4N and
// N_cp <= N/4: one wavefront per Doppler row, every transform a pair of
// 32-point DFT passes done as matrix products.
//
// Per Doppler row s with taps u[n], n < N_cp:
//   X_k  = sum_n u[n] W_N^{k n}                          (forward DFT_N)
//   G_b[q] = sum_k w_k X_k V_{4N}^{k b} V_N^{k q}         (b = 1, 2, 3)
//   P[s][4q + b] = |G_b[q]|^2 / (N M)
// with W_L = e^{-2 pi i/L}, V_L = e^{+2 pi i/L}; phase b = 0 is the three-tap
// filter of the taps (IDFT_N of a cosine window has three taps).
//
// Both N-point transforms split their indices 32 x 32 (the Cooley-Tukey
// factorisation), with n = n_a + 32 n_b (n_b < 8 since N_cp <= 256),
// k = k_a + 32 k_b and q = q_a + 32 q_b:
//   f1  Y[k_a][n_a]  = sum_{n_b} W_32^{k_a n_b} u[n_a + 32 n_b]
//   t1  Y'           = Y W_N^{k_a n_a}
//   f2  X[k_a+32k_b] = sum_{n_a} W_32^{k_b n_a} Y'[k_a][n_a]
//   i1  Z[k_a][q_a]  = sum_{k_b} V_32^{k_b q_a} X_b[k_a + 32 k_b],  X_b = w_k V_{4N}^{k b} X_k
//   t2  Z'           = Z V_N^{k_a q_a}
//   i2  G_b[q_a+32q_b] = sum_{k_a} V_32^{k_a q_b} Z'[k_a][q_a]
// Each pass is a real 64 x 64 (or 16 x 64) product of a constant DFT matrix
// with the row's data, on v_mfma_f32_32x32x16 with operands split into two
// half-precision parts (v = hi + lo, hi = rn(v), lo = rn(v - hi); the
// products lo*hi, hi*lo and hi*hi accumulate in FP32), or in the FP16 form
// rounded once to FP16 with one product per pass (about 2^-11 relative per
// operand instead of 2^-22, for a third of the matrix-core work).
//
// Fragment layouts of v_mfma_f32_32x32x16 (lane l, i = l % 32, h = l / 32):
//   A (32 x 16): lane l holds A[i][8h + e], e < 8
//   B (16 x 32): lane l holds B[8h + e][i], e < 8
//   C (32 x 32): lane l holds C[mx_row(h, e)][i], e < 16,
//                mx_row(h, e) = 8 (e / 4) + 4h + e % 4
// A pass that takes the data as A leaves the data's row index in the result
// rows (registers) and puts the constant's column index in the lanes; a pass
// that takes it as B keeps its column (lane) index.  Alternating the two --
// f1 as A, f2 as B, i1 as A, i2 as B -- contracts each index where it sits,
// so no lane exchange is needed anywhere: a lane holds column i of every
// result, and the index in its 16 rows always matches the K layout of the
// next pass once that pass's constant has its K index permuted to match.
// A result's rows (re in one 32-row block, im in the other) feed the next
// pass's K-block q as [re of rows 4q..4q+3 | im of rows 4q..4q+3]: element j
// of lane half h is (part j / 4, index 8q + 4h + j % 4).
//
// The inverse constant serves all three inverse passes: i1's B fragment and
// i2's A fragment hold the same values in every lane, and f2 computes
// conj(sum V conj(Y')) with it (the conjugations fold into the twiddle
// products on either side).
//
// Range of the half-precision operands: each row is scaled by a power of two
// s so that its largest tap component lies in [2^12, 2^13); the twiddles of
// t1 and t2 carry 2^-3 and the phase factors 2^-5, so every operand stays
// below 2^15.5 (worst case, all terms in phase) while the FP32 accumulators
// take the growth of each pass.  P is rescaled by the exact power of two.
#pragma once

#include "mfma_dft.hpp"

namespace radar {

__device__ __forceinline__ constexpr int mx_row(int h, int e) { return 8 * (e >> 2) + 4 * h + (e & 3); }

typedef uint32_t mx_u32x4 __attribute__((ext_vector_type(4)));

// The lane index, opaque to the optimiser (an empty asm statement emits no
// instruction): table reads indexed by it are issued where they are used
// instead of being hoisted and held in registers across the row.
__device__ __forceinline__ int mx_opaque(int v) {
  asm volatile("" : "+v"(v));
  return v & 63;
}

// (a, b) -> packed hi = rn(a, b) and lo = rn(a - hi_a, b - hi_b) in halves
template <Prec P>
struct MxSplit;

template <>
struct MxSplit<Prec::FP16X3> {
  // lo by one mixed-precision FMA per value, reading hi as a half and the
  // value as a float: the difference is exact inside the FMA and rounded once
  static __device__ __forceinline__ void pair(float a, float b, uint32_t& hi, uint32_t& lo) {
    typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
    const h2_t h = __builtin_convertvector(f32x2_t{a, b}, h2_t);
    hi = __builtin_bit_cast(uint32_t, h);
    uint32_t l;
    asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(l) : "v"(hi), "v"(a));
    asm("v_fma_mixhi_f16 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(l) : "v"(hi), "v"(b));
    lo = l;
  }
};

// FP16 rounded once: the lo part is not formed
template <>
struct MxSplit<Prec::FP16> {
  static __device__ __forceinline__ void pair(float a, float b, uint32_t& hi, uint32_t& lo) {
    typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
    hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{a, b}, h2_t));
    lo = 0u;
  }
};

template <>
struct MxSplit<Prec::BF16X3> {
  static __device__ __forceinline__ void pair(float a, float b, uint32_t& hi, uint32_t& lo) {
    typedef __bf16 b2_t __attribute__((ext_vector_type(2)));
    const f32x2_t v{a, b};
    const b2_t h = __builtin_convertvector(v, b2_t);
    const f32x2_t r = v - __builtin_convertvector(h, f32x2_t);
    hi = __builtin_bit_cast(uint32_t, h);
    lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, b2_t));
  }
};

// One K-block operand (8 values per lane), split.
template <Prec P>
struct MxFrag {
  using vec8 = typename PrecTraits<P>::vec8;
  vec8 hi, lo;
  __device__ __forceinline__ void set(const float (&v)[8]) {
    mx_u32x4 h, l;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t x, y;
      MxSplit<P>::pair(v[2 * j], v[2 * j + 1], x, y);
      h[j] = x;
      l[j] = y;
    }
    hi = __builtin_bit_cast(vec8, h);
    lo = __builtin_bit_cast(vec8, l);
  }
};

// c + a b with both operands split: lo*hi, hi*lo, then hi*hi; the FP16 form
// (operands rounded once) takes hi*hi alone
template <Prec P>
__device__ __forceinline__ f32x16_t mma3(const MxFrag<P>& a, const MxFrag<P>& b, f32x16_t c) {
  if constexpr (P != Prec::FP16) {
    c = PrecTraits<P>::mfma(a.lo, b.hi, c);
    c = PrecTraits<P>::mfma(a.hi, b.lo, c);
  }
  return PrecTraits<P>::mfma(a.hi, b.hi, c);
}

// K-block q of the next pass from a result held as (re[16], im[16])
template <Prec P>
__device__ __forceinline__ MxFrag<P> mx_kblock(const float (&re)[16], const float (&im)[16], int q) {
  float v[8];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    v[j] = re[4 * q + j];
    v[4 + j] = im[4 * q + j];
  }
  MxFrag<P> f;
  f.set(v);
  return f;
}

template <int N>
struct K3Mx {
  static_assert(N == 1024, "the matrix-core range stage factors N as 32 x 32");
  static constexpr int WAVES = 8;  // two waves per SIMD: one's vector work overlaps the other's products
  static constexpr int BLOCK = 64 * WAVES;
  static constexpr int UB = N / 4 + 3;  // taps u[-1 .. N/4+1] per wave (phase 0)
};

// The persistent range kernel on the matrix cores.  kStore = false keeps
// only the row maxima; kRefs takes P row pointers from the batch job table.
// Held in registers across rows: the inverse 32-point DFT fragments (i1's B,
// i2's A, f2's A).  In LDS, read per row: f1's B fragments, the twiddles
// W_N^{i mx_row} 2^-3 of t1 and t2, and the phase factors.
template <int N, Prec PR, bool kStore = true, bool kRefs = false>
__global__ void __launch_bounds__(K3Mx<N>::BLOCK) k3_range_power_mx(K3Args a, int total_rows) {
  using C = K3Mx<N>;
  using Frag = MxFrag<PR>;
  using vec8 = typename PrecTraits<PR>::vec8;
  constexpr int Q = N / 4;
  __shared__ float2 s_ph[3 * 16 * 64];        // w_k V_{4N}^{k b} 2^-5 as [b-1][e][lane]
  __shared__ float2 s_tw[16 * 64];            // W_N^{i mx_row(h, e)} 2^-3 as [e][lane]
  __shared__ vec8 s_f1[2][2][64];             // f1's B fragments [ob][hi, lo][lane]
  __shared__ float2 s_ub[C::WAVES][C::UB];    // each wave's taps, unscaled
  __shared__ float s_p[C::WAVES][2][16][64];  // phases 1 and 2 of the row until phase 3 joins them

  const int lane = threadIdx.x & 63;
  const int i = lane & 31, h = lane >> 5;
  const float2 wc = window_coeffs(a.window);
  {
    constexpr int poff = phase_offset(ilog2c(N), 2);
    for (int idx = threadIdx.x; idx < 3 * 16 * 64; idx += C::BLOCK) {
      const int b = (idx >> 10) + 1, e = (idx >> 6) & 15, l = idx & 63;
      const int k = (l & 31) + 32 * mx_row(l >> 5, e);
      const float w = (wc.x - wc.y * g_radar_tw[(unsigned)(N + k)].x) * 0.03125f;
      const float2 t = g_radar_tw[(unsigned)(poff + b * N + k)];  // W_{4N}^{k b}
      s_ph[idx] = make_float2(w * t.x, -w * t.y);
    }
    for (int idx = threadIdx.x; idx < 16 * 64; idx += C::BLOCK) {
      const int e = idx >> 6, l = idx & 63;
      s_tw[idx] = cscale(g_radar_tw[(unsigned)(N + (((l & 31) * mx_row(l >> 5, e)) & (N - 1)))], 0.125f);
    }
    if (threadIdx.x < 128) {
      // B[8h + e][i] of f1: (part h, n_b = e) against column k_a = i, W_32^{n_b k_a}
      const int ob = threadIdx.x >> 6;
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float2 w = g_radar_tw[(unsigned)(32 + ((e * i) & 31))];
        v[e] = ob == 0 ? (h == 0 ? w.x : -w.y) : (h == 0 ? w.y : w.x);
      }
      Frag f;
      f.set(v);
      s_f1[ob][0][lane] = f.hi;
      s_f1[ob][1][lane] = f.lo;
    }
  }
  // the inverse 32-point DFT fragments of this lane: (part, x) of element e
  // of K-block q is (e / 4, 8q + 4h + e % 4), value V_32^{x i} by the rule
  // re-out: (re v, -im v), im-out: (im v, re v) over (part re, part im)
  Frag vc[2][4];
#pragma unroll
  for (int ob = 0; ob < 2; ++ob)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int x = 8 * q + 4 * h + (e & 3);
        const float2 w = g_radar_tw[(unsigned)(32 + ((x * i) & 31))];
        const float vr = w.x, vi = -w.y;  // V_32^{x i}
        v[e] = ob == 0 ? ((e >> 2) == 0 ? vr : -vi) : ((e >> 2) == 0 ? vi : vr);
      }
      vc[ob][q].set(v);
    }

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float2* ub = s_ub[wave] + 1;
  if (lane < 3) ub[lane == 0 ? -1 : Q + lane - 1] = make_float2(0.0f, 0.0f);
  const float c0 = (float)N * wc.x * sqrtf(a.scale), c1 = -0.5f * (float)N * wc.y * sqrtf(a.scale);
  __syncthreads();

  // lane (i, h) holds part h (re, im) of u[i + 32 e], e < 8
  auto load_taps = [&](float (&uv)[8], int grow) {
    const RADAR_GLOBAL float* src = gptr(reinterpret_cast<const float*>(a.U + (int64_t)grow * a.n_cp));
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int n = i + 32 * e;
      uv[e] = n < a.n_cp ? src[2 * n + h] : 0.0f;
    }
  };
  const int stride = gridDim.x * C::WAVES;
  float uv[8];
  int grow = blockIdx.x * C::WAVES + wave;
  if (grow < total_rows) load_taps(uv, grow);
  for (; grow < total_rows; grow += stride) {
    const int f = grow / a.m_pad;
    const int row = grow - f * a.m_pad;
    // the row's scale: its largest tap component to [2^12, 2^13)
    float mu = 0.0f;
#pragma unroll
    for (int e = 0; e < 8; ++e) mu = fmaxf(mu, fabsf(uv[e]));
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) mu = fmaxf(mu, __shfl_xor(mu, m));
    int ex = 0;
    frexpf(mu, &ex);
    ex = mu > 0.0f ? (ex < -100 ? -100 : ex) : 0;
    const float sc = ldexpf(1.0f, 13 - ex);
    const float cp = ldexpf(a.scale, 2 * ex - 4);  // P = |G_s|^2 / (N M) (2^13 / s)^2
    // taps to LDS for phase 0
#pragma unroll
    for (int e = 0; e < 8; ++e) reinterpret_cast<float*>(ub)[2 * (i + 32 * e) + h] = uv[e];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // read by other lanes in the epilogue

    // f1: data as A (K: part h, n_b = e), W_32 as B
    f32x16_t y0, y1;
    {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = uv[e] * sc;
      Frag d;
      d.set(v);
      Frag b0, b1;
      b0.hi = s_f1[0][0][lane];
      b0.lo = s_f1[0][1][lane];
      b1.hi = s_f1[1][0][lane];
      b1.lo = s_f1[1][1][lane];
      y0 = mma3<PR>(d, b0, f32x16_t{});
      y1 = mma3<PR>(d, b1, f32x16_t{});
    }
    // t1, conjugated for f2: conj(Y W_N^{k_a n_a} 2^-3)
    f32x16_t x0{}, x1{};
    {
      float re[16], im[16];
      const int ln = mx_opaque(lane);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const float2 t = s_tw[e * 64 + ln];
        re[e] = y0[e] * t.x - y1[e] * t.y;
        im[e] = -(y0[e] * t.y + y1[e] * t.x);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const Frag d = mx_kblock<PR>(re, im, q);
        x0 = mma3<PR>(vc[0][q], d, x0);
        x1 = mma3<PR>(vc[1][q], d, x1);
      }
    }
    // (x0, x1) = conj(X 2^-3), X[i + 32 mx_row(h, e)].  Phases 1..3 in turn:
    // X_b = X w V_{4N}^{k b} 2^-5; i1 with X_b as A; t2 (Z V_N^{k_a q_a} 2^-3,
    // k_a = mx_row, q_a = i); i2 with Z' as B; |.|^2
    const int gnext = grow + stride;
    float un[8];
    RADAR_GLOBAL float* dst = nullptr;
    if constexpr (kStore) {
      const auto* crefs = (const __attribute__((address_space(4))) FrameRef*)a.refs;
      dst = gptr(kRefs ? crefs[f].P : a.P + (int64_t)f * a.p_stride) + (int64_t)row * (4 * N);
    }
    float mx = 0.0f;
    float mg = 0.0f;  // without stores: the largest |G|^2 of phases 1..3, unscaled
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      f32x16_t z0{}, z1{};
      {
        float re[16], im[16];
        const int ln = mx_opaque(lane);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const float2 p = s_ph[(b * 16 + e) * 64 + ln];
          re[e] = x0[e] * p.x + x1[e] * p.y;
          im[e] = x0[e] * p.y - x1[e] * p.x;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const Frag d = mx_kblock<PR>(re, im, q);
          z0 = mma3<PR>(d, vc[0][q], z0);
          z1 = mma3<PR>(d, vc[1][q], z1);
        }
      }
      f32x16_t g0{}, g1{};
      {
        float re[16], im[16];
        const int ln = mx_opaque(lane);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const float2 t = s_tw[e * 64 + ln];
          re[e] = z0[e] * t.x + z1[e] * t.y;
          im[e] = z1[e] * t.x - z0[e] * t.y;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const Frag d = mx_kblock<PR>(re, im, q);
          g0 = mma3<PR>(vc[0][q], d, g0);
          g1 = mma3<PR>(vc[1][q], d, g1);
        }
      }
      if (!kStore) {
        // only the maximum is kept: scaling by cp > 0 is monotone, so it is
        // applied once to the largest |G|^2
#pragma unroll
        for (int e = 0; e < 16; ++e) mg = fmaxf(mg, g0[e] * g0[e] + g1[e] * g1[e]);
        if (b == 2) {
          if (gnext < total_rows) load_taps(un, gnext);
          mx = mg * cp;
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            const int r1 = i + 32 * mx_row(h, e);
            if (mx_row(h, e) <= Q / 32) {
              if (r1 <= Q)
                mx = fmaxf(mx, cabs2(cadd(cscale(ub[r1], c0), cscale(cadd(ub[r1 - 1], ub[r1 + 1]), c1))));
            } else if (mx_row(h, e) == 31) {
              if (i == 31) mx = fmaxf(mx, cabs2(cscale(ub[0], c1)));
            }
          }
        }
      } else if (b < 2) {
#pragma unroll
        for (int e = 0; e < 16; ++e) s_p[wave][b][e][lane] = (g0[e] * g0[e] + g1[e] * g1[e]) * cp;
      } else {
        // the next row's taps, loaded before this row's stores so that
        // waiting for them does not wait for the stores
        if (gnext < total_rows) load_taps(un, gnext);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const float p1 = s_p[wave][0][e][lane], p2 = s_p[wave][1][e][lane];
          const float p3 = (g0[e] * g0[e] + g1[e] * g1[e]) * cp;
          const int r1 = i + 32 * mx_row(h, e);
          // phase 0: the three-tap filter where the taps reach (r1 <= N/4, and the wrap r1 = N - 1)
          float p0 = 0.0f;
          if (mx_row(h, e) <= Q / 32) {
            if (r1 <= Q) p0 = cabs2(cadd(cscale(ub[r1], c0), cscale(cadd(ub[r1 - 1], ub[r1 + 1]), c1)));
          } else if (mx_row(h, e) == 31) {
            if (i == 31) p0 = cabs2(cscale(ub[0], c1));
          }
          if constexpr (kStore)
            __builtin_nontemporal_store(radar_v4{p0, p1, p2, p3}, (RADAR_GLOBAL radar_v4*)(dst + 4 * r1));
          mx = fmaxf(fmaxf(fmaxf(fmaxf(mx, p0), p1), p2), p3);
        }
      }
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
    if (lane == 0) a.rowmax[grow] = mx;
#pragma unroll
    for (int e = 0; e < 8; ++e) uv[e] = un[e];
    // the next row's tap writes must follow this row's reads of ub
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

}  // namespace radar
