// The CNN sub-cell refiner: patch extraction, forward, backward and Adam.
//
// Network (48 576 parameters, flat FP32 master vector in this order):
//   conv1 3x3 1->32 s1, conv2 3x3 32->32 s2, conv3 3x3 32->32 s1, conv4 3x3 32->32 s2
//   (weights [co][ky][kx][ci], biases [co], zero padding 1, ReLU),
//   fc1 2048->10 (weights [10][2048] over the NHWC flattening (y*8+x)*32+c, ReLU),
//   fc2 10->2.
// Activations are NHWC with 32 channels, stored in BF16; gradients in FP32.
//
// The three 32->32 convolutions run on the matrix cores as implicit GEMMs
// (k_conv_mfma): for the forward pass C[co][pixel] = sum_K W[co][K] X[K][pixel]
// with K = tap * 32 + ci, so one lane's 8 operand values are 8 consecutive
// channels of one NHWC pixel (a 16-byte load); the input gradient is the same
// product with the roles of ci and co exchanged, gathered from the output
// gradient.  conv1 (one input channel), the weight gradients, the dense layers
// and Adam are FP32 vector kernels.
#pragma once

#include "device_common.hpp"
#include "mfma_dft.hpp"

namespace radar {

constexpr int kCnnParams = 48576;
constexpr int kOffConv1W = 0, kOffConv1B = 288;
constexpr int kOffConv2W = 320, kOffConv2B = 320 + 9216;
constexpr int kOffConv3W = kOffConv2B + 32, kOffConv3B = kOffConv3W + 9216;
constexpr int kOffConv4W = kOffConv3B + 32, kOffConv4B = kOffConv4W + 9216;
constexpr int kOffFc1W = kOffConv4B + 32, kOffFc1B = kOffFc1W + 20480;
constexpr int kOffFc2W = kOffFc1B + 10, kOffFc2B = kOffFc2W + 20;
static_assert(kOffFc2B + 2 == kCnnParams, "parameter layout");

__device__ __forceinline__ float bf2f(__bf16 v) { return (float)v; }

// FP32 conv2..conv4 weights -> BF16 copies (3 x 9216, [co][tap][ci])
__global__ void k_cnn_weights_bf16(const float* theta, __bf16* wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * 9216) return;
  const int layer = i / 9216, j = i - layer * 9216;
  const int off = layer == 0 ? kOffConv2W : (layer == 1 ? kOffConv3W : kOffConv4W);
  wb[i] = (__bf16)theta[off + j];
}

// ---------------------------------------------------------------- patches
// Patch n = f * k + i: the 32 x 32 window of frame f's P centred on peak i,
// ln(max(P, 1e-12 P_c)) - ln P_c (cyclic in both axes); valid[n] = 0 when
// frame f has fewer than i + 1 peaks (the patch is then zero).
__global__ void __launch_bounds__(256) k_cnn_patches(const float* P, int64_t p_stride, int m_pad, int n_pad, int k,
                                                     const radar_peak* peaks, const int32_t* n_peaks, float* out,
                                                     int32_t* valid) {
  const int n = blockIdx.x;
  const int f = n / k, i = n - f * k;
  const bool ok = i < n_peaks[f];
  const radar_peak pk = peaks[n];
  const int row = ok ? pk.s + m_pad / 2 : 0;
  const int col = ok ? pk.r : 0;
  const float* base = P + (int64_t)f * p_stride;
  const float pc = ok ? base[(int64_t)row * n_pad + col] : 1.0f;
  const float lpc = logf(pc);
  for (int t = threadIdx.x; t < 1024; t += 256) {
    const int y = t >> 5, x = t & 31;
    const int rr = (row + y - 16) & (m_pad - 1), cc = (col + x - 16) & (n_pad - 1);
    const float v = ok ? base[(int64_t)rr * n_pad + cc] : pc;
    out[(int64_t)n * 1024 + t] = ok ? logf(fmaxf(v, 1e-12f * pc)) - lpc : 0.0f;
  }
  if (threadIdx.x == 0 && valid) valid[n] = ok ? 1 : 0;
}

// ------------------------------------------------------------ conv1 (VALU)
// One thread per output pixel (b, y, x): 32 channels, ReLU, BF16 NHWC.
__global__ void __launch_bounds__(256) k_conv1_fwd(const float* x, const float* theta, __bf16* a1, int B) {
  __shared__ float w[288 + 32];
  for (int i = threadIdx.x; i < 320; i += 256) w[i] = theta[kOffConv1W + i];
  __syncthreads();
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= B * 1024) return;
  const int b = p >> 10, y = (p >> 5) & 31, xx = p & 31;
  float in[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int iy = y + t / 3 - 1, ix = xx + t % 3 - 1;
    in[t] = (iy >= 0 && iy < 32 && ix >= 0 && ix < 32) ? x[((int64_t)b << 10) + iy * 32 + ix] : 0.0f;
  }
  __bf16* o = a1 + (int64_t)p * 32;
#pragma unroll
  for (int co = 0; co < 32; ++co) {
    float z = w[288 + co];
#pragma unroll
    for (int t = 0; t < 9; ++t) z = fmaf(w[co * 9 + t], in[t], z);
    o[co] = (__bf16)fmaxf(z, 0.0f);
  }
}

// ------------------------------------------------- 32->32 conv on the MFMA
// MODE 0 (forward): in = activations x [B][H][W][32] (BF16), out = relu(conv) [B][H/S][W/S][32] (BF16).
// MODE 1 (input gradient): in = dz [B][H/S][W/S][32] (FP32), out = dx * (a_prev > 0) [B][H][W][32]
// (FP32, a_prev the layer's input activations: the ReLU of the layer below).
// One wave computes a 32-channel x 32-pixel tile with 18 MFMAs (K = 288).
template <int S, int MODE>
__global__ void __launch_bounds__(256) k_conv_mfma(const void* in_, const __bf16* wb, const float* bias,
                                                   const __bf16* a_prev, void* out_, int B, int H, int W) {
  const int Ho = H / S, Wo = W / S;
  const int lane = threadIdx.x & 63, h = lane >> 5, i = lane & 31;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  // output pixels of this tile: forward over (b, oy, ox), gradient over (b, iy, ix)
  const int OH = MODE == 0 ? Ho : H, OW = MODE == 0 ? Wo : W;
  const int total = B * OH * OW;
  const int p = wave * 32 + i;
  if (wave * 32 >= total) return;  // whole wave beyond the last tile (total is a multiple of 32)
  const int b = p / (OH * OW), rem = p - b * OH * OW;
  const int py = rem / OW, px = rem - py * OW;

  // A fragments for all 18 K slices: forward A[co][K] = W[co][tap][ci];
  // gradient A[ci][K] = W[co][tap][ci] with K = tap * 32 + co
  bf16x8_t a[18];
#pragma unroll
  for (int q = 0; q < 18; ++q) {
    const int tap = q >> 1, c0 = 16 * (q & 1) + 8 * h;
    if constexpr (MODE == 0) {
      a[q] = *reinterpret_cast<const bf16x8_t*>(wb + (i * 9 + tap) * 32 + c0);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) a[q][e] = wb[((c0 + e) * 9 + tap) * 32 + i];
    }
  }
  f32x16_t c = {};
#pragma unroll
  for (int q = 0; q < 18; ++q) {
    const int tap = q >> 1, ky = tap / 3, kx = tap - ky * 3, c0 = 16 * (q & 1) + 8 * h;
    bf16x8_t bv;
    if constexpr (MODE == 0) {
      const int iy = S * py + ky - 1, ix = S * px + kx - 1;
      if (iy >= 0 && iy < H && ix >= 0 && ix < W) {
        const __bf16* src = static_cast<const __bf16*>(in_) + (((int64_t)b * H + iy) * W + ix) * 32 + c0;
        bv = *reinterpret_cast<const bf16x8_t*>(src);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[e] = (__bf16)0.0f;
      }
    } else {
      const int ty = py + 1 - ky, tx = px + 1 - kx;  // = S * oy, S * ox
      const int oy = ty / S, ox = tx / S;
      const bool okp = ty >= 0 && tx >= 0 && oy * S == ty && ox * S == tx && oy < Ho && ox < Wo;
      if (okp) {
        const float* src = static_cast<const float*>(in_) + (((int64_t)b * Ho + oy) * Wo + ox) * 32 + c0;
        const float4 u0 = *reinterpret_cast<const float4*>(src);
        const float4 u1 = *reinterpret_cast<const float4*>(src + 4);
        bv[0] = (__bf16)u0.x; bv[1] = (__bf16)u0.y; bv[2] = (__bf16)u0.z; bv[3] = (__bf16)u0.w;
        bv[4] = (__bf16)u1.x; bv[5] = (__bf16)u1.y; bv[6] = (__bf16)u1.z; bv[7] = (__bf16)u1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[e] = (__bf16)0.0f;
      }
    }
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[q], bv, c, 0, 0, 0);
  }
  // lane holds rows (channels) 8 g + 4 h + j, j < 4, of column (pixel) p
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int ch = 8 * g + 4 * h;
    if constexpr (MODE == 0) {
      __bf16* dst = static_cast<__bf16*>(out_) + (int64_t)p * 32 + ch;
#pragma unroll
      for (int j = 0; j < 4; ++j) dst[j] = (__bf16)fmaxf(c[4 * g + j] + bias[ch + j], 0.0f);
    } else {
      const __bf16* ap = a_prev + (int64_t)p * 32 + ch;
      float4 v;
      v.x = bf2f(ap[0]) > 0.0f ? c[4 * g + 0] : 0.0f;
      v.y = bf2f(ap[1]) > 0.0f ? c[4 * g + 1] : 0.0f;
      v.z = bf2f(ap[2]) > 0.0f ? c[4 * g + 2] : 0.0f;
      v.w = bf2f(ap[3]) > 0.0f ? c[4 * g + 3] : 0.0f;
      *reinterpret_cast<float4*>(static_cast<float*>(out_) + (int64_t)p * 32 + ch) = v;
    }
  }
}

// ----------------------------------------------------- weight gradients
// Per image: dW[co][tap][ci] = sum_pix dz[pix][co] x[in(pix, tap)][ci] and
// db[co] = sum_pix dz[pix][co] (32 -> 32 layers, x BF16, dz FP32), partial
// sums per image in part[b][9248] (weights then biases).
template <int S>
__global__ void __launch_bounds__(256) k_conv_wgrad(const __bf16* x, const float* dz, float* part, int H, int W) {
  extern __shared__ float smem[];
  const int Ho = H / S, Wo = W / S;
  const int HP = H + 2, WP = W + 2;
  float* sdz = smem;                                               // [Ho*Wo][32]
  __bf16* sx = reinterpret_cast<__bf16*>(smem + Ho * Wo * 32);     // [HP][WP][32], zero border
  const int b = blockIdx.x;
  for (int t = threadIdx.x; t < Ho * Wo * 32; t += 256) sdz[t] = dz[(int64_t)b * Ho * Wo * 32 + t];
  for (int t = threadIdx.x; t < HP * WP * 32; t += 256) {
    const int c = t & 31, pix = t >> 5, yy = pix / WP - 1, xx = pix % WP - 1;
    sx[t] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? x[(((int64_t)b * H + yy) * W + xx) * 32 + c]
                                                     : (__bf16)0.0f;
  }
  __syncthreads();
  const int co = threadIdx.x >> 3, ci0 = (threadIdx.x & 7) * 4;
  float acc[9][4] = {};
  float accb = 0.0f;
  for (int pix = 0; pix < Ho * Wo; ++pix) {
    const int oy = pix / Wo, ox = pix - oy * Wo;
    const float d = sdz[pix * 32 + co];
    accb += d;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const __bf16* xs = sx + ((S * oy + tap / 3) * WP + S * ox + tap % 3) * 32 + ci0;
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[tap][j] = fmaf(d, bf2f(xs[j]), acc[tap][j]);
    }
  }
  float* dst = part + (int64_t)b * 9248;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[(co * 9 + tap) * 32 + ci0 + j] = acc[tap][j];
  if ((threadIdx.x & 7) == 0) dst[9216 + co] = accb;
}

// conv1: part[b][320] = dW1[co][tap] (288) then db1[co] (32), x the FP32 input patch
__global__ void __launch_bounds__(256) k_conv1_wgrad(const float* x, const float* dz, float* part) {
  __shared__ float sx[34 * 34];
  __shared__ float red[8][320];
  const int b = blockIdx.x;
  for (int t = threadIdx.x; t < 34 * 34; t += 256) {
    const int yy = t / 34 - 1, xx = t % 34 - 1;
    sx[t] = (yy >= 0 && yy < 32 && xx >= 0 && xx < 32) ? x[((int64_t)b << 10) + yy * 32 + xx] : 0.0f;
  }
  __syncthreads();
  const int co = threadIdx.x & 31, grp = threadIdx.x >> 5;
  float acc[9] = {}, accb = 0.0f;
  for (int pix = grp; pix < 1024; pix += 8) {
    const float d = dz[(((int64_t)b << 10) + pix) * 32 + co];
    const int y = pix >> 5, xx = pix & 31;
    accb += d;
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = fmaf(d, sx[(y + t / 3) * 34 + xx + t % 3], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 9; ++t) red[grp][co * 9 + t] = acc[t];
  red[grp][288 + co] = accb;
  __syncthreads();
  for (int t = threadIdx.x; t < 320; t += 256) {
    float s = 0.0f;
#pragma unroll
    for (int g = 0; g < 8; ++g) s += red[g][t];
    part[(int64_t)b * 320 + t] = s;
  }
}

// grad[off + j] = sum_b part[b][j], j < n (the per-image partials summed in image order)
__global__ void k_sum_partials(const float* part, int nb, int n, float* grad, int off) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float s = 0.0f;
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * n + j];
  grad[off + j] = s;
}

// ---------------------------------------------------------- dense layers
// One work-group per patch: fc1 (2048 -> 10, ReLU) and fc2 (10 -> 2).
__global__ void __launch_bounds__(256) k_fc_fwd(const __bf16* a4, const float* theta, float* z5, float* out) {
  __shared__ float red[10][4];
  __shared__ float a5[10];
  const int b = blockIdx.x;
  const __bf16* xin = a4 + (int64_t)b * 2048;
  float acc[10] = {};
  for (int i = threadIdx.x; i < 2048; i += 256) {
    const float v = bf2f(xin[i]);
#pragma unroll
    for (int j = 0; j < 10; ++j) acc[j] = fmaf(theta[kOffFc1W + j * 2048 + i], v, acc[j]);
  }
#pragma unroll
  for (int j = 0; j < 10; ++j) {
    float v = acc[j];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    if ((threadIdx.x & 63) == 0) red[j][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 10) {
    const int j = threadIdx.x;
    const float z = red[j][0] + red[j][1] + red[j][2] + red[j][3] + theta[kOffFc1B + j];
    z5[b * 10 + j] = z;
    a5[j] = fmaxf(z, 0.0f);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int o = threadIdx.x;
    float s = theta[kOffFc2B + o];
#pragma unroll
    for (int j = 0; j < 10; ++j) s = fmaf(theta[kOffFc2W + o * 10 + j], a5[j], s);
    out[b * 2 + o] = s;
  }
}

// Mean squared error over the batch and both outputs: dout = 2 (out - label) / (2 B);
// loss[0] = the mean (one work-group).
__global__ void __launch_bounds__(256) k_mse(const float* out, const float* label, int B, float* dout, float* loss) {
  __shared__ float red[4];
  float acc = 0.0f;
  const float sc = 2.0f / (2.0f * (float)B);
  for (int i = threadIdx.x; i < 2 * B; i += 256) {
    const float d = out[i] - label[i];
    dout[i] = sc * d;
    acc += d * d;
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) loss[0] = (red[0] + red[1] + red[2] + red[3]) / (2.0f * (float)B);
}

// dz5 = (dout W2) * (z5 > 0) per patch, and the fc2 gradients (one work-group).
__global__ void __launch_bounds__(256) k_fc2_bwd(const float* dout, const float* z5, const float* theta, int B,
                                                 float* dz5, float* grad) {
  __shared__ float red[4][22];
  float acc[22] = {};
  for (int b = threadIdx.x; b < B; b += 256) {
    float a5[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) a5[j] = fmaxf(z5[b * 10 + j], 0.0f);
    const float d0 = dout[2 * b], d1 = dout[2 * b + 1];
#pragma unroll
    for (int j = 0; j < 10; ++j) {
      acc[j] = fmaf(d0, a5[j], acc[j]);
      acc[10 + j] = fmaf(d1, a5[j], acc[10 + j]);
      const float da = d0 * theta[kOffFc2W + j] + d1 * theta[kOffFc2W + 10 + j];
      dz5[b * 10 + j] = z5[b * 10 + j] > 0.0f ? da : 0.0f;
    }
    acc[20] += d0;
    acc[21] += d1;
  }
#pragma unroll
  for (int q = 0; q < 22; ++q) {
    float v = acc[q];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < 22) {
    const float s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
    grad[threadIdx.x < 20 ? kOffFc2W + threadIdx.x : kOffFc2B + threadIdx.x - 20] = s;
  }
}

// fc1 gradients: thread per weight (j, i) summing over the batch, plus biases.
__global__ void __launch_bounds__(256) k_fc1_wgrad(const __bf16* a4, const float* dz5, int B, float* grad) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < 20480) {
    const int j = t / 2048, i = t - j * 2048;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s = fmaf(dz5[b * 10 + j], bf2f(a4[(int64_t)b * 2048 + i]), s);
    grad[kOffFc1W + t] = s;
  } else if (t < 20490) {
    const int j = t - 20480;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += dz5[b * 10 + j];
    grad[kOffFc1B + j] = s;
  }
}

// dz4[b][i] = (sum_j dz5[b][j] W1[j][i]) * (a4[b][i] > 0)
__global__ void __launch_bounds__(256) k_fc1_dgrad(const __bf16* a4, const float* dz5, const float* theta, int B,
                                                   float* dz4) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)B * 2048) return;
  const int b = (int)(t >> 11), i = (int)(t & 2047);
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 10; ++j) s = fmaf(dz5[b * 10 + j], theta[kOffFc1W + j * 2048 + i], s);
  dz4[t] = bf2f(a4[t]) > 0.0f ? s : 0.0f;
}

// ------------------------------------------------- fused inference kernel
// The whole network for one patch per work-group iteration, every activation
// resident in LDS (BF16, NHWC, zero halo for the next layer's padding) and
// every weight resident in registers across patches:
//   s_in [34][34] FP32 input, s_a1 [34][34][CP], s_a2 [18][18][CP],
//   s_a3 [18][18][CP], s_a4 [8][8][32]; pixels CP = 40 channels (80 bytes, an
//   odd multiple of 16) apart, so the 16-byte operand reads of 16 consecutive
//   pixels fall in distinct bank groups (2-way for the stride-2 layers).
// Four waves, one per SIMD.  conv1 runs on the matrix cores too: K = 9 taps
// padded to 16, with the input and weights split into BF16 hi + lo parts
// (hi*hi + hi*lo + lo*hi in FP32), so its outputs match an FP32 convolution
// to about 2^-16.  conv2..conv4 are 32-channel x 32-pixel tiles, two per wave
// at a time (independent accumulators hide the MFMA latency).  The dense layers
// are work-group reductions with each thread's slice of the 2048 -> 10 weights in
// registers.  Persistent: work-group b takes patches b, b + gridDim.x, ...;
// only the patch (4 KB) and the two outputs touch HBM.
constexpr int kFusedThreads = 256;
struct FusedLds {
  static constexpr int CP = 40;                 // channel stride of the padded activations
  static constexpr int IN = 34 * 34;            // floats
  static constexpr int A1 = 34 * 34 * CP;       // bf16
  static constexpr int A2 = 18 * 18 * CP;
  static constexpr int A3 = 18 * 18 * CP;
  static constexpr int A4 = 8 * 8 * 32;
  static constexpr size_t BYTES = IN * 4 + (size_t)(A1 + A2 + A3 + A4) * 2 + 4 * 11 * 4;
};

// 18 A fragments of one 32->32 layer (W[co][tap][ci], co = lane % 32)
__device__ __forceinline__ void load_conv_frags(bf16x8_t (&a)[18], const __bf16* wb, int h, int i) {
#pragma unroll
  for (int q = 0; q < 18; ++q) {
    const int tap = q >> 1, c0 = 16 * (q & 1) + 8 * h;
    a[q] = *reinterpret_cast<const bf16x8_t*>(wb + (i * 9 + tap) * 32 + c0);
  }
}

// Two 32-channel x 32-pixel tiles (pixels (oy0, ox0) and (oy1, ox1) of this
// lane's column) of a 32->32 convolution from an LDS input with WP columns.
template <int S>
__device__ __forceinline__ void conv_tiles_lds(const __bf16* src, int WP, int oy0, int ox0, int oy1, int ox1,
                                               const bf16x8_t (&a)[18], int h, f32x16_t& c0, f32x16_t& c1) {
  c0 = {};
  c1 = {};
#pragma unroll
  for (int q = 0; q < 18; ++q) {
    const int tap = q >> 1, ky = tap / 3, kx = tap - ky * 3, ch = 16 * (q & 1) + 8 * h;
    const bf16x8_t b0 =
        *reinterpret_cast<const bf16x8_t*>(src + ((S * oy0 + ky) * WP + S * ox0 + kx) * FusedLds::CP + ch);
    const bf16x8_t b1 =
        *reinterpret_cast<const bf16x8_t*>(src + ((S * oy1 + ky) * WP + S * ox1 + kx) * FusedLds::CP + ch);
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[q], b0, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[q], b1, c1, 0, 0, 0);
  }
}

// bias + ReLU of a tile into a BF16 NHWC destination pixel
__device__ __forceinline__ void store_tile(const f32x16_t& c, const float* bias, __bf16* dst, int h) {
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int ch = 8 * g + 4 * h;
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[ch + j] = (__bf16)fmaxf(c[4 * g + j] + bias[ch + j], 0.0f);
  }
}

__global__ void __launch_bounds__(kFusedThreads) k_cnn_fused(const float* x, const float* theta, const __bf16* wb,
                                                             int B, float* out) {
  extern __shared__ float fsm[];
  float* s_in = fsm;
  __bf16* s_a1 = reinterpret_cast<__bf16*>(s_in + FusedLds::IN);
  __bf16* s_a2 = s_a1 + FusedLds::A1;
  __bf16* s_a3 = s_a2 + FusedLds::A2;
  __bf16* s_a4 = s_a3 + FusedLds::A3;
  float* s_red = reinterpret_cast<float*>(s_a4 + FusedLds::A4);  // [4 waves][11]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, i = lane & 31;
  // zero every buffer once: the halos stay zero, interiors are rewritten per patch
  for (int t = tid; t < FusedLds::IN; t += kFusedThreads) s_in[t] = 0.0f;
  for (int t = tid; t < FusedLds::A1 + FusedLds::A2 + FusedLds::A3 + FusedLds::A4; t += kFusedThreads)
    s_a1[t] = (__bf16)0.0f;
  // weights, kept in registers for every patch
  bf16x8_t w1h, w1l;  // conv1 as A[co][tap], taps 9..15 zero
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int tap = 8 * h + e;
    const float v = tap < 9 ? theta[kOffConv1W + i * 9 + tap] : 0.0f;
    const __bf16 hi = (__bf16)v;
    w1h[e] = hi;
    w1l[e] = (__bf16)(v - (float)hi);
  }
  bf16x8_t a2[18], a3[18], a4[18];
  load_conv_frags(a2, wb, h, i);
  load_conv_frags(a3, wb + 9216, h, i);
  load_conv_frags(a4, wb + 2 * 9216, h, i);
  float wf[8][10];  // dense 2048 -> 10: inputs tid + 256 r, r < 8
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int j = 0; j < 10; ++j) wf[r][j] = theta[kOffFc1W + j * 2048 + tid + 256 * r];
  __syncthreads();

  for (int p = blockIdx.x; p < B; p += gridDim.x) {
    const float* xp = x + (int64_t)p * 1024;
    for (int t = tid; t < 1024; t += kFusedThreads) s_in[((t >> 5) + 1) * 34 + (t & 31) + 1] = xp[t];
    __syncthreads();
    // conv1: 32 tiles of 32 pixels, 8 per wave; B[tap][pixel] = input shifted by the tap
#pragma unroll 2
    for (int tt = 0; tt < 8; ++tt) {
      const int pix = (wave * 8 + tt) * 32 + i, y = pix >> 5, xx = pix & 31;
      bf16x8_t bh, bl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int tap = 8 * h + e;
        const float v = tap < 9 ? s_in[(y + tap / 3) * 34 + xx + tap % 3] : 0.0f;
        const __bf16 hi = (__bf16)v;
        bh[e] = hi;
        bl[e] = (__bf16)(v - (float)hi);
      }
      f32x16_t c = {};
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1l, bh, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1h, bl, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1h, bh, c, 0, 0, 0);
      store_tile(c, theta + kOffConv1B, s_a1 + ((y + 1) * 34 + xx + 1) * FusedLds::CP, h);
    }
    __syncthreads();
    f32x16_t c0, c1;
    // conv2: 32x32 -> 16x16, 8 tiles, two per wave
    {
      const int p0 = (2 * wave) * 32 + i, p1 = p0 + 32;
      conv_tiles_lds<2>(s_a1, 34, p0 >> 4, p0 & 15, p1 >> 4, p1 & 15, a2, h, c0, c1);
      store_tile(c0, theta + kOffConv2B, s_a2 + (((p0 >> 4) + 1) * 18 + (p0 & 15) + 1) * FusedLds::CP, h);
      store_tile(c1, theta + kOffConv2B, s_a2 + (((p1 >> 4) + 1) * 18 + (p1 & 15) + 1) * FusedLds::CP, h);
    }
    __syncthreads();
    // conv3: 16x16 -> 16x16
    {
      const int p0 = (2 * wave) * 32 + i, p1 = p0 + 32;
      conv_tiles_lds<1>(s_a2, 18, p0 >> 4, p0 & 15, p1 >> 4, p1 & 15, a3, h, c0, c1);
      store_tile(c0, theta + kOffConv3B, s_a3 + (((p0 >> 4) + 1) * 18 + (p0 & 15) + 1) * FusedLds::CP, h);
      store_tile(c1, theta + kOffConv3B, s_a3 + (((p1 >> 4) + 1) * 18 + (p1 & 15) + 1) * FusedLds::CP, h);
    }
    __syncthreads();
    // conv4: 16x16 -> 8x8, 2 tiles (wave 0)
    if (wave == 0) {
      const int p0 = i, p1 = 32 + i;
      conv_tiles_lds<2>(s_a3, 18, p0 >> 3, p0 & 7, p1 >> 3, p1 & 7, a4, h, c0, c1);
      store_tile(c0, theta + kOffConv4B, s_a4 + p0 * 32, h);
      store_tile(c1, theta + kOffConv4B, s_a4 + p1 * 32, h);
    }
    __syncthreads();
    // dense 2048 -> 10 (ReLU) -> 2
    float acc[10] = {};
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const float v = bf2f(s_a4[tid + 256 * r]);
#pragma unroll
      for (int j = 0; j < 10; ++j) acc[j] = fmaf(wf[r][j], v, acc[j]);
    }
#pragma unroll
    for (int j = 0; j < 10; ++j) {
      float v = acc[j];
#pragma unroll
      for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
      if (lane == 0) s_red[wave * 11 + j] = v;
    }
    __syncthreads();
    if (tid < 2) {
      float o = theta[kOffFc2B + tid];
#pragma unroll
      for (int j = 0; j < 10; ++j) {
        const float z = theta[kOffFc1B + j] + s_red[j] + s_red[11 + j] + s_red[22 + j] + s_red[33 + j];
        o = fmaf(theta[kOffFc2W + tid * 10 + j], fmaxf(z, 0.0f), o);
      }
      out[(int64_t)p * 2 + tid] = o;
    }
    __syncthreads();  // s_in and s_red are rewritten for the next patch
  }
}

// -------------------------------------------------------------------- Adam
// omb1 = 1 - b1 and omb2 = 1 - b2 are rounded once from exact values (1 - 0.999f
// in FP32 would carry a 1.3e-5 relative error into every second moment).
__global__ void k_adam(float* theta, const float* grad, float* m, float* v, int n, float lr, float b1, float b2,
                       float omb1, float omb2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + omb1 * g;
  const float vi = b2 * v[i] + omb2 * g * g;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);  // c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t)
}

}  // namespace radar
