// Split-precision 16-point DFTs on the matrix cores: the precision form of
// the radix-16 FFT stages.
//
// One wavefront transforms 64 independent 16-point columns at once, each lane
// holding its own column x[0..15] on entry and its 16 outputs on return (the
// same contract as the FP32 in-register DFT).  In real arithmetic the DFT of a
// block of 32 columns is one 32 x 32 by 32 x 32 product:
//     [Yr; Yi] = A1 Xr + A2 Xi,   A1 = [Fr; Fi],  A2 = [-Fi; Fr],
// F = Fr + i Fi the 16 x 16 DFT matrix.  Each operand is split into two
// half-precision parts, v = v_hi + v_lo with v_hi = rn(v) and
// v_lo = rn(v - v_hi), and the three products hi*hi, hi*lo and lo*hi are
// accumulated in FP32 by v_mfma_f32_32x32x16 (the lo*lo term is below the
// FP32 rounding of the result).  BF16 keeps FP32's exponent range; FP16 has
// three more mantissa bits but a narrow range, so each column is scaled by a
// power of two that puts its largest component in [2^14, 2^15) before the
// split and unscaled afterwards (exact).
//
// Fragment layouts of v_mfma_f32_32x32x16 (lane l, h = l / 32, i = l % 32):
//   A (32 x 16): lane l holds A[i][8h + e], e < 8
//   B (16 x 32): lane l holds B[8h + e][i], e < 8
//   C (32 x 32): lane l holds C[8 (e / 4) + 4h + e % 4][i], e < 16
// Column block 0 holds the columns of lanes 0..31 and block 1 those of lanes
// 32..63; v_permlane32_swap moves the column halves into place on the way in
// and the output halves back to their column's lane on the way out.
#pragma once

#include "fft.hpp"

namespace radar {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// FP16: FP16 operands rounded once (no split), one product per pass; only
// the matrix-core range stage implements it.
enum class Prec { FP32 = 0, BF16X3 = 1, FP16X3 = 2, FP16 = 3 };

template <Prec P>
struct PrecTraits;

template <>
struct PrecTraits<Prec::BF16X3> {
  using half_t = __bf16;
  using vec8 = bf16x8_t;
  static constexpr bool kScale = false;
  static __device__ __forceinline__ f32x16_t mfma(vec8 a, vec8 b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct PrecTraits<Prec::FP16> {
  using half_t = _Float16;
  using vec8 = f16x8_t;
  static constexpr bool kScale = true;
  static __device__ __forceinline__ f32x16_t mfma(vec8 a, vec8 b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct PrecTraits<Prec::FP16X3> {
  using half_t = _Float16;
  using vec8 = f16x8_t;
  static constexpr bool kScale = true;
  static __device__ __forceinline__ f32x16_t mfma(vec8 a, vec8 b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

typedef float f32x2_t __attribute__((ext_vector_type(2)));

// v = hi + lo with hi = rn(v), lo = rn(v - hi), into element e of two vectors
template <class V>
__device__ __forceinline__ void split_into(float v, V& hi, V& lo, int e) {
  using H = decltype(hi[0] + hi[0]);
  const H h = (H)v;
  hi[e] = h;
  lo[e] = (H)(v - (float)h);
}

// The same for the pair (a, b) into elements e, e + 1 (e even): one packed
// conversion per part.
template <class V>
__device__ __forceinline__ void split_pair(float a, float b, V& hi, V& lo, int e) {
  using H = decltype(hi[0] + hi[0]);
  typedef H h2_t __attribute__((ext_vector_type(2)));
  const f32x2_t v = {a, b};
  const h2_t h = __builtin_convertvector(v, h2_t);
  const f32x2_t r = v - __builtin_convertvector(h, f32x2_t);
  const h2_t l = __builtin_convertvector(r, h2_t);
  hi[e] = h[0];
  hi[e + 1] = h[1];
  lo[e] = l[0];
  lo[e + 1] = l[1];
}

template <Prec P>
struct DftMfma {
  using Tr = PrecTraits<P>;
  using vec8 = typename Tr::vec8;
  static constexpr bool kWave = true;  // every lane of the wavefront must call run<16>
  // A1/A2 fragments of the forward DFT matrix, hi and lo parts.  The inverse
  // DFT is swap(DFT(swap(x))) with swap(a + ib) = b + ia (= i conj), which
  // only exchanges the roles of the real and imaginary registers.
  vec8 f1h, f1l, f2h, f2l;

  __device__ __forceinline__ void init() {
    const int l = threadIdx.x & 63;
    const int i = l & 31, h = l >> 5;
    const int row = i & 15;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int q = (row * (8 * h + e)) & 15;
      const float c = Tw16::c[q], s = Tw16::s[q];
      // F = cos - i sin: A1 = [Fr; Fi], A2 = [-Fi; Fr]
      const float f1 = i < 16 ? c : -s, f2 = i < 16 ? s : c;
      split_into(f1, f1h, f1l, e);
      split_into(f2, f2h, f2l, e);
    }
  }

  template <int R, bool INV>
  __device__ __forceinline__ void run(float2* x) const {
    if constexpr (R != 16) {
      Dft<R, INV>::run(x);
    } else {
      run16<INV>(x);
    }
  }

  template <bool INV>
  __device__ __forceinline__ void run16(float2* x) const {
    float sc = 1.0f;
    if constexpr (Tr::kScale) {
      float mx = 0.0f;
#pragma unroll
      for (int e = 0; e < 16; ++e) mx = fmaxf(mx, fmaxf(fabsf(x[e].x), fabsf(x[e].y)));
      int ex = 0;
      frexpf(mx, &ex);  // mx in [2^(ex-1), 2^ex)
      ex = ex < -100 ? -100 : ex;  // keep 1/sc a normal float for (near-)zero columns
      sc = mx > 0.0f ? ldexpf(1.0f, 15 - ex) : 1.0f;
    }
    // H0 = x[0..7], H1 = x[8..15].  Swapping the upper 32 lanes of H0 with the
    // lower 32 lanes of H1 leaves in H0 the B operand of column block 0
    // (rows 0..7 of columns 0..31 in lanes 0..31, rows 8..15 in lanes 32..63)
    // and in H1 that of block 1.
    float2 b0[8], b1[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float xr = INV ? x[e].y : x[e].x, xi = INV ? x[e].x : x[e].y;
      const float yr = INV ? x[8 + e].y : x[8 + e].x, yi = INV ? x[8 + e].x : x[8 + e].y;
      const auto re = __builtin_amdgcn_permlane32_swap(__float_as_uint(xr * sc), __float_as_uint(yr * sc), false,
                                                       false);
      const auto im = __builtin_amdgcn_permlane32_swap(__float_as_uint(xi * sc), __float_as_uint(yi * sc), false,
                                                       false);
      b0[e] = make_float2(__uint_as_float(re[0]), __uint_as_float(im[0]));
      b1[e] = make_float2(__uint_as_float(re[1]), __uint_as_float(im[1]));
    }
    f32x16_t acc[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      vec8 rh, rl, ih, il;
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        const float2 v = cb == 0 ? b0[e] : b1[e];
        const float2 w = cb == 0 ? b0[e + 1] : b1[e + 1];
        split_pair(v.x, w.x, rh, rl, e);
        split_pair(v.y, w.y, ih, il, e);
      }
      f32x16_t c = {};
      c = Tr::mfma(f1l, rh, c);
      c = Tr::mfma(f2l, ih, c);
      c = Tr::mfma(f1h, rl, c);
      c = Tr::mfma(f2h, il, c);
      c = Tr::mfma(f1h, rh, c);
      c = Tr::mfma(f2h, ih, c);
      acc[cb] = c;
    }
    // Lane l holds rows 8(e/4) + 4h + e%4 of column l % 32 of each block.  The
    // same swap on the two accumulators leaves in o0 the outputs 0..3, 8..11
    // and in o1 the outputs 4..7, 12..15 of the lane's own column.
    const float isc = 1.0f / sc;
    float o0[16], o1[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc[0][e]), __float_as_uint(acc[1][e]),
                                                      false, false);
      o0[e] = __uint_as_float(r[0]) * isc;
      o1[e] = __uint_as_float(r[1]) * isc;
    }
    // elements 0..7 hold real parts, 8..15 imaginary parts (swapped back for the inverse)
    auto cx = [](float re, float im) { return INV ? make_float2(im, re) : make_float2(re, im); };
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x[j] = cx(o0[j], o0[8 + j]);
      x[8 + j] = cx(o0[4 + j], o0[12 + j]);
      x[4 + j] = cx(o1[j], o1[8 + j]);
      x[12 + j] = cx(o1[4 + j], o1[12 + j]);
    }
  }
};

template <Prec P>
struct DftFor {
  using type = DftMfma<P>;
};
template <>
struct DftFor<Prec::FP32> {
  using type = DftFp32;
};

}  // namespace radar
