// Peak search without a materialised periodogram (P = NULL): the range
// kernel kept only the row maxima, k_peak_threshold listed the rows that can
// hold a top-k local maximum, and this kernel recomputes, for each listed
// row, that row and its two cyclic neighbours into LDS with the range
// kernel's own row code, then scans the row exactly as k_peak_rows_listed
// scans a row of P.  The row code is compiled into this kernel too, and the
// compiler may order a few multiply-adds differently here: a recomputed cell
// can differ from the one the range kernel writes by a few FP32 ulps.
#pragma once

#include "k_frame.hpp"
#include "k_peaks.hpp"

namespace radar {

// LDS of the recompute kernel (256 threads, float2 units): the range
// kernel's tables, then one exchange region and one tap buffer per computing
// team, then the three rows (4N floats each).  The scan's n_pad = 4N words of
// candidate marks reuse the exchange regions once the rows are done.
template <int N>
struct K3Recompute {
  using C = K3p<N>;
  static constexpr int T = C::T;
  static constexpr int BLOCK = 256;
  static constexpr int WAVES = (3 * T + 63) / 64;       // waves holding teams 0, 1, 2
  static constexpr int TEAMS = WAVES * 64 / T;          // teams in those waves
  static constexpr int XCH = C::TAB;
  static constexpr int UB = XCH + TEAMS * C::EXCH;
  static constexpr int ROWS = (UB + TEAMS * C::UBUF + 1) & ~1;  // 16-byte aligned
  static constexpr int POOL = ROWS + 3 * (4 * N) / 2;
  static_assert(TEAMS * C::EXCH * 2 >= 4 * N, "scan marks fit the exchange regions");
  static_assert(WAVES * 64 <= BLOCK, "computing waves");
};

// Grid (G, F), 256 threads.  For list entry j of frame f (row s): teams 0, 1
// and 2 compute rows s-1, s and s+1; other teams of their waves compute row s
// again and keep nothing (no divergence inside a wave); the remaining waves
// only scan.  Output cand[f][j][0..k) as k_peak_rows_listed.
template <int N, Prec PR>
__global__ void __launch_bounds__(256) k_peak_rows_recompute(K3Args a, int k, const float* tau, const int32_t* list,
                                                             const int32_t* cnt, uint64_t* cand) {
  using C = K3p<N>;
  using R = K3Recompute<N>;
  constexpr int T = C::T;
  constexpr int NP = 4 * N;
  typename DftFor<PR>::type df;
  df.init();
  __shared__ __align__(16) float2 pool[R::POOL];
  __shared__ uint64_t red[4];
  __shared__ int s_cnt[4];
  float2* const tab = pool;
  const float2 cf = k3p_tables<N>(tab, a.window, a.scale, threadIdx.x, R::BLOCK);
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool computes = wave < R::WAVES;                  // wave-uniform
  const int g = threadIdx.x / T;                          // team
  const int gc = g < R::TEAMS ? g : 0;
  const int t = threadIdx.x - g * T;
  float2* lds = pool + R::XCH + gc * C::EXCH;
  float2* ub = pool + R::UB + gc * C::UBUF + 1;           // ub[i] = u[i], i in [-1, N/4+1]
  float* rows = reinterpret_cast<float*>(pool + R::ROWS);  // rows s-1, s, s+1
  uint32_t* s_ord = reinterpret_cast<uint32_t*>(pool + R::XCH);

  const int f = blockIdx.y;
  const int count = cnt[f];
  const float th = tau[f];
  const int mask = a.m_pad - 1;
  for (int j = blockIdx.x; j < count; j += gridDim.x) {
    const int row = list[(int64_t)f * a.m_pad + j];
    if (computes) {
      const int rr = (row + (g < 3 ? g - 1 : 0)) & mask;
      float2 uv[4];
      k3p_load_taps<N>(uv, a.U + ((int64_t)f * a.m_pad + rr) * a.n_cp, a.n_cp, t);
      k3p_put_taps<N>(ub, uv, a.n_cp, t);
      k3p_zero_pads<N>(ub, t);
      const RowToLds sink{g < 3 ? rows + g * NP : nullptr};
      (void)k3p_row<N, PR>(lds, ub, t, tab, cf.x, cf.y, df, sink, [] {});
    }
    __syncthreads();  // the rows are complete; the exchange regions are free for the marks
    row_candidates(static_cast<const float*>(rows), static_cast<const float*>(rows + NP),
                   static_cast<const float*>(rows + 2 * NP), NP, k, th, (uint32_t)row * (uint32_t)NP, s_ord, red,
                   s_cnt, cand + ((int64_t)f * a.m_pad + j) * k);
    // row_candidates ends with a barrier: the next entry may overwrite the rows
  }
}

}  // namespace radar
