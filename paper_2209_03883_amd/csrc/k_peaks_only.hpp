// Peak search without a materialised periodogram (P = NULL): the range
// kernel kept only the row maxima, k_peak_threshold listed the rows that can
// hold a top-k local maximum (ascending), and k_peak_rows_window recomputes
// the rows a scan needs with the range kernel's own row code, then scans
// each listed row exactly as k_peak_rows_listed scans a row of P.  The row
// code is compiled into this kernel too, and the compiler may order a few
// multiply-adds differently here: a recomputed cell can differ from the one
// the range kernel writes by a few FP32 ulps.
//
// Listed rows come in runs of neighbours (a strong target's Doppler main lobe
// and side lobes span many rows), so each wavefront walks a contiguous share
// of the list and computes the union of {s-1, s, s+1} over its entries in
// ascending order, every row once: a run of L listed rows costs L + 2 row
// transforms, not 3 L.  The rows go to a small per-wavefront ring in global
// memory (read back at once, from the caches) and each entry is scanned by
// its wavefront alone as soon as its row s+1 is done, with no work-group
// barrier after the tables are built.
#pragma once

#include "k_frame.hpp"
#include "k_peaks.hpp"

namespace radar {

// A ring row in global memory: plain (cached) stores, since the same
// wavefront reads the row back within microseconds.
struct RowToRing {
  RADAR_GLOBAL float* dst;
  __device__ __forceinline__ void store4(int i, float a, float b, float c, float d) const {
    gstore4(dst + i, a, b, c, d);
  }
  __device__ __forceinline__ void store2(int i, float a, float b) const { gstore2(dst + i, a, b); }
};

// One listed row by one wavefront (no barriers; every lane must call it):
// its exact local maxima >= th among the rows above (rm), at (r0) and below
// (rp), NP = n_pad columns, cyclic.  The k best keys go to out[0..k) (key 0
// pads), as row_candidates leaves them.  Lane l owns the column groups
// 8 (l + 64 q) .. +7, q < NP / 512: its candidates are one bit each in a
// 64-bit mask, and values are read again from the ring (cache hits) when the
// keys are formed.
template <int NP>
__device__ __forceinline__ void wave_row_candidates(const RADAR_GLOBAL float* rm, const RADAR_GLOBAL float* r0,
                                                    const RADAR_GLOBAL float* rp, int k, float th, uint32_t flat0,
                                                    uint64_t* out, int lane) {
  constexpr int Q = NP / 512;
  static_assert(Q >= 1 && Q <= 8 && NP == 512 * Q, "eight columns per lane per group, at most 64 per lane");
  uint64_t bits = 0;
#pragma unroll 4
  for (int q = 0; q < Q; ++q) {
    const int c0 = 8 * (lane + 64 * q);
    float a[3][10];
    load_cols10(rm, c0, NP, a[0]);
    load_cols10(r0, c0, NP, a[1]);
    load_cols10(rp, c0, NP, a[2]);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float v = a[1][u + 1];
      bool pk = v >= th;
#pragma unroll
      for (int d = 0; d < 3; ++d) pk = pk && v >= a[0][u + d] && v >= a[2][u + d];
      pk = pk && v >= a[1][u] && v >= a[1][u + 2];
      bits |= pk ? 1ull << (8 * q + u) : 0ull;
    }
  }
  const int mine = __popcll(bits);
  int incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int up = __shfl_up(incl, off);
    if (lane >= off) incl += up;
  }
  const int total = __shfl(incl, 63);
  const auto col_of = [&](int i) { return 8 * (lane + 64 * (i >> 3)) + (i & 7); };
  if (total <= k) {
    // few candidates: all of them (the merge ranks), then 0 pads
    int pos = incl - mine;
    for (uint64_t b = bits; b; b &= b - 1) {
      const int c = col_of(__builtin_ctzll(b));
      out[pos++] = make_key(ord_bits(r0[c]), flat0 + (uint32_t)c);
    }
    for (int q = total + lane; q < k; q += 64) out[q] = 0;
  } else {
    // k rounds of "largest key below the previous one" over the wavefront
    uint64_t last = ~0ull;
    for (int i = 0; i < k; ++i) {
      uint64_t best = 0;
      for (uint64_t b = bits; b; b &= b - 1) {
        const int c = col_of(__builtin_ctzll(b));
        const uint64_t key = make_key(ord_bits(r0[c]), flat0 + (uint32_t)c);
        if (key < last && key > best) best = key;
      }
      best = wave_max_u64(best);
      if (lane == 0) out[i] = best;
      last = best;
    }
  }
}

// The recompute kernel's shape: the range kernel's work-group (8 wavefronts,
// ROWS = 64 / T teams each, one row per team per step) and LDS pool; each
// wavefront's ring holds RING = ROWS + 2 rows of n_pad = 4N floats (a step's
// ROWS new rows and the two before them, which the first entry scanned in
// the step may need).
template <int N>
struct K3Window {
  using C = K3p<N>;
  static constexpr int RING = C::ROWS + 2;
  static constexpr size_t kRingFloatsPerBlock = (size_t)C::WAVES * RING * 4 * N;
};

// Grid (G_total), K3p<N>::BLOCK threads; work items (frame f, share gs) for
// f < n_frames, gs < per_frame, taken in turn by the work-groups.  The
// wavefronts of a work-group split the item's share of frame f's list
// entries [start[f] (0 without start), cnt[f]) into contiguous pieces, each
// ascending.  Output cand[f][j][0..k) for every such entry j, as
// k_peak_rows_listed.  ring: gridDim.x * kRingFloatsPerBlock floats.
template <int N, Prec PR>
__global__ void __launch_bounds__(K3p<N>::BLOCK) k_peak_rows_window(K3Args a, int n_frames, int per_frame, int k,
                                                                    const float* tau, const int32_t* list,
                                                                    const int32_t* cnt, const int32_t* start,
                                                                    uint64_t* cand, float* ring) {
  using C = K3p<N>;
  using W = K3Window<N>;
  constexpr int T = C::T;
  constexpr int R = C::ROWS;
  constexpr int NP = 4 * N;
  constexpr int kNone = -0x40000000;  // no row (below any row index, less one)
  const int items = n_frames * per_frame;
  // a work-group whose frames have no entries in range leaves before building
  // its tables (the second listing usually adds none); the test depends on
  // blockIdx only, so the whole work-group leaves together
  {
    bool any = false;
    for (int item = blockIdx.x; item < items && !any; item += gridDim.x) {
      const int f = item / per_frame;
      any = cnt[f] > (start ? start[f] : 0);
    }
    if (!any) return;
  }
  typename DftFor<PR>::type df;
  df.init();
  __shared__ float2 pool[C::TAB + C::WAVES * C::ROWS * (C::EXCH + C::UBUF)];
  float2* const tab = pool;
  auto xch = reinterpret_cast<float2 (*)[C::ROWS][C::EXCH]>(pool + C::TAB);
  auto ubuf = reinterpret_cast<float2 (*)[C::ROWS][C::UBUF]>(pool + C::TAB + C::WAVES * C::ROWS * C::EXCH);
  const float2 cf = k3p_tables<N>(tab, a.window, a.scale, threadIdx.x, C::BLOCK);
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int g = lane / T;
  const int t0 = lane - g * T;
  float2* lds = xch[wave][g];
  float2* ub = ubuf[wave][g] + 1;  // ub[i] = u[i], i in [-1, N/4+1]
  k3p_zero_pads<N>(ub, t0);
  RADAR_GLOBAL float* const my_ring = gptr(ring) + ((size_t)blockIdx.x * C::WAVES + wave) * (W::RING * NP);
  const int mask = a.m_pad - 1;

  __shared__ int s_sum[C::WAVES];
  __shared__ int s_piece[C::WAVES][2];
  const int tid = threadIdx.x;
  // work-group sum of one value per thread (every thread gets it)
  const auto block_sum = [&](int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) s_sum[wave] = v;
    __syncthreads();
    int t = 0;
#pragma unroll
    for (int w = 0; w < C::WAVES; ++w) t += s_sum[w];
    __syncthreads();
    return t;
  };

  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int f = item / per_frame;
    const int share = item - f * per_frame;
    const int j0 = start ? start[f] : 0;
    const int count = cnt[f] - j0;
    if (count <= 0) continue;  // work-group-uniform
    const int32_t* L = list + (int64_t)f * a.m_pad;
    // Pieces of equal work: entry j adds min(3, s_j - s_{j-1}) rows to the
    // union (3 for the first), and the frame's pieces split the running
    // total evenly; this work-group's wavefronts take pieces share * WAVES +
    // wave.  Entries stay in order, so each piece is a contiguous range.
    const auto cost = [&](int j) {
      if (j == 0) return 3;
      const int d = L[j0 + j] - L[j0 + j - 1];
      return d < 3 ? d : 3;
    };
    int part = 0;
    for (int j = tid; j < count; j += C::BLOCK) part += cost(j);
    const int64_t total = block_sum(part);
    const int pieces = per_frame * C::WAVES;
    if (tid < C::WAVES) {
      s_piece[tid][0] = count;
      s_piece[tid][1] = 0;
    }
    int run = 0;  // the union rows of the entries before this chunk
    for (int base = 0; base < count; base += C::BLOCK) {
      const int j = base + tid;
      const int c = j < count ? cost(j) : 0;
      int incl = c;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int up = __shfl_up(incl, off);
        if (lane >= off) incl += up;
      }
      if (lane == 63) s_sum[wave] = incl;
      __syncthreads();  // also orders this chunk's s_piece updates after the initialisation
      int before = 0, chunk = 0;
#pragma unroll
      for (int w = 0; w < C::WAVES; ++w) {
        before += w < wave ? s_sum[w] : 0;
        chunk += s_sum[w];
      }
      if (j < count) {
        const int64_t excl = run + before + incl - c;
        const int q = (int)(excl * pieces / total) - share * C::WAVES;
        if (q >= 0 && q < C::WAVES) {
          atomicMin(&s_piece[q][0], j);
          atomicMax(&s_piece[q][1], j + 1);
        }
      }
      run += chunk;
      __syncthreads();  // s_sum is reused by the next chunk
    }
    const int ja = j0 + s_piece[wave][0];
    const int jb = j0 + s_piece[wave][1];
    if (ja >= jb) continue;  // wave-uniform
    const float th = tau[f];
    const float2* Uf = a.U + (int64_t)f * a.m_pad * a.n_cp;

    // the union of {s-1, s, s+1} over entries ja .. jb-1, ascending, each
    // row once (rows -1 and m_pad stand for m_pad-1 and 0)
    int e = ja, prev = kNone;
    const auto gen = [&]() -> int {
      while (e < jb) {
        const int s = L[e];
        const int r = s - 1 > prev + 1 ? s - 1 : prev + 1;
        if (r <= s + 1) {
          prev = r;
          return r;
        }
        ++e;
      }
      return kNone;
    };
    const auto pick = [&](const int (&rows)[R]) {  // this team's row of a step (team 0's where it has none)
      int r = rows[0];
#pragma unroll
      for (int q = 1; q < R; ++q)
        if (g == q && rows[q] != kNone) r = rows[q];
      return r;
    };
    int cur[R], nxt[R];
#pragma unroll
    for (int q = 0; q < R; ++q) cur[q] = gen();
#pragma unroll
    for (int q = 0; q < R; ++q) nxt[q] = gen();
    float2 uv[4];
    k3p_load_taps<N>(uv, Uf + (int64_t)(pick(cur) & mask) * a.n_cp, a.n_cp, t0);
    k3p_put_taps<N>(ub, uv, a.n_cp, t0);

    int ubase = 0;  // union index of this step's first row
    int js = ja;    // next entry to scan
    while (true) {
      // the opaque team lane of the range kernel (addresses formed again per row)
      int t = t0;
      if constexpr (K3pOrder<N, PR>::kOneStore) {
        asm volatile("" : "+v"(t));
        t &= T - 1;
      }
      const bool more = nxt[0] != kNone;
      const int rn = pick(nxt);
      const auto next = [&] {
        if (more) k3p_load_taps<N>(uv, Uf + (int64_t)(rn & mask) * a.n_cp, a.n_cp, t);
      };
      const RowToRing sink{my_ring + (size_t)((ubase + g) % W::RING) * NP};
      (void)k3p_row<N, PR>(lds, ub, t, tab, cf.x, cf.y, df, sink, next);
      // the next row's tap writes must follow this row's reads of ub
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      if (more) k3p_put_taps<N>(ub, uv, a.n_cp, t);
      // the ring rows of every team are complete and visible to the whole wavefront
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");

      int nvalid = 0, last = kNone;
#pragma unroll
      for (int q = 0; q < R; ++q)
        if (cur[q] != kNone) ++nvalid, last = cur[q];
      // every entry whose row s+1 came in this step: rows s-1, s, s+1 are
      // union indices u-2, u-1, u (no union row lies between them)
      while (js < jb && L[js] + 1 <= last) {
        const int s = L[js];
        int u = ubase;
#pragma unroll
        for (int q = 1; q < R; ++q)
          if (cur[q] == s + 1) u = ubase + q;
        const RADAR_GLOBAL float* rm = my_ring + (size_t)((u - 2) % W::RING) * NP;
        const RADAR_GLOBAL float* r0 = my_ring + (size_t)((u - 1) % W::RING) * NP;
        const RADAR_GLOBAL float* rp = my_ring + (size_t)(u % W::RING) * NP;
        wave_row_candidates<NP>(rm, r0, rp, k, th, (uint32_t)s * (uint32_t)NP,
                                cand + ((int64_t)f * a.m_pad + js) * k, lane);
        ++js;
      }
      ubase += nvalid;
      if (!more) break;
#pragma unroll
      for (int q = 0; q < R; ++q) cur[q] = nxt[q];
#pragma unroll
      for (int q = 0; q < R; ++q) nxt[q] = gen();
    }
  }
}

}  // namespace radar
