// Register/LDS Stockham FFT used by every radar kernel.
//
// A transform of length L (a power of two) is computed by a "team" of
// T = L/E threads; each thread holds E complex values (E = 4, 8 or 16) in
// registers in the cyclic layout  v[e] = x[t + T*e].  The transform runs as a
// sequence of Stockham stages of radix E (and one final stage of a smaller
// radix when L is not a power of E).  Between stages the team exchanges data
// through its own LDS region; the last stage leaves its outputs in
// registers, again in the cyclic layout, so X[t + T*e] = v[e] on return and
// natural order needs no final reordering.
//
// Stage s with radix R and span NS (the product of the earlier radices):
// butterfly j in [0, L/R) reads x[j + m*L/R] (m < R), multiplies element m by
// W_{NS*R}^{(j mod NS)*m}, runs an R-point DFT and writes output m to
// position (j - j mod NS)*R + (j mod NS) + m*NS.
//
// Forward transforms use exp(-2 pi i nk/L); INV transforms use exp(+2 pi i nk/L)
// without the 1/L factor.
#pragma once

#include <utility>

#include "device_common.hpp"

namespace radar {

// cos(2 pi q/16) and sin(2 pi q/16), q = 0..15.
struct Tw16 {
  static constexpr float c[16] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
  static constexpr float s[16] = {
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};
};

// a * exp(-2 pi i Q/16) (forward) or a * exp(+2 pi i Q/16) (INV).
template <int Q, bool INV>
__device__ __forceinline__ float2 rot16(float2 a) {
  constexpr int q = Q & 15;
  if constexpr (q == 0) {
    return a;
  } else if constexpr (q == 4) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
  } else if constexpr (q == 8) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (q == 12) {
    return INV ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
  } else {
    constexpr float c = Tw16::c[q];
    constexpr float s = Tw16::s[q];
    if constexpr (INV) {
      return make_float2(a.x * c - a.y * s, a.y * c + a.x * s);
    } else {
      return make_float2(a.x * c + a.y * s, a.y * c - a.x * s);
    }
  }
}

// In-register R-point DFT (R = 1, 2, 4, 8, 16), decimation in time.
template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<1, INV> {
  static __device__ __forceinline__ void run(float2*) {}
};

template <int R, bool INV, int K>
__device__ __forceinline__ void dit_combine_one(float2* x, const float2* e, const float2* o) {
  const float2 t = rot16<K * (16 / R), INV>(o[K]);
  x[K] = cadd(e[K], t);
  x[K + R / 2] = csub(e[K], t);
}

template <int R, bool INV, int... K>
__device__ __forceinline__ void dit_combine(float2* x, const float2* e, const float2* o,
                                            std::integer_sequence<int, K...>) {
  (dit_combine_one<R, INV, K>(x, e, o), ...);
}

template <int R, bool INV>
struct Dft {
  static_assert(R == 2 || R == 4 || R == 8 || R == 16, "radix");
  static __device__ __forceinline__ void run(float2* x) {
    float2 e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    Dft<R / 2, INV>::run(e);
    Dft<R / 2, INV>::run(o);
    dit_combine<R, INV>(x, e, o, std::make_integer_sequence<int, R / 2>{});
  }
};

// The FP32 in-register DFT of a Stockham stage (the plain form); other
// policies (the matrix-core form) provide the same run<R, INV>().  A policy
// with kWave = true must be called by every lane of the wavefront.
struct DftFp32 {
  static constexpr bool kWave = false;
  __device__ __forceinline__ void init() {}
  template <int R, bool INV>
  __device__ __forceinline__ void run(float2* x) const {
    Dft<R, INV>::run(x);
  }
};

// LDS index with one pad slot every 16 entries (limits bank conflicts of the
// strided Stockham writes).
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }
template <int L>
struct LdsSize {
  static constexpr int value = L + L / 16;
};

// Synchronisation of one team around an LDS exchange.  A team inside one
// wavefront only needs its LDS writes to land before its reads: the LDS
// serves a wave's instructions in order, so a compiler-level fence plus a wait
// for the wave's own LDS operations suffices and leaves global loads in
// flight.  Wider teams use the work-group barrier.
template <int T>
__device__ __forceinline__ void team_sync() {
  if constexpr (T <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Where a stage's twiddles come from: the global stage section, or a copy of
// the stages a kernel needs in LDS (Layout::off<NS, R>() gives each block's
// offset there, same [m][k] layout).
struct TwGlobal {
  template <int NS, int R>
  __device__ __forceinline__ float2 stage(int k, int m) const {
    return stage_twiddle<NS, R>(k, m);
  }
};

template <class Layout>
struct TwLds {
  const float2* base;
  template <int NS, int R>
  __device__ __forceinline__ float2 stage(int k, int m) const {
    return base[Layout::template off<NS, R>() + m * NS + k];
  }
};

// The same LDS copy, but a stage's twiddles are read after the exchange
// rather than before it: the prefetch then holds no registers across the
// exchange (for kernels that keep much else live through the transform).
template <class Layout>
struct TwLdsLate : TwLds<Layout> {};

template <class TS>
struct TwFetchLate {
  static constexpr bool value = false;
};
template <class Layout>
struct TwFetchLate<TwLdsLate<Layout>> {
  static constexpr bool value = true;
};

// Shape of the Stockham stage that starts at span NS.
template <int L, int E, int NS>
struct StagePlan {
  static constexpr int T = L / E;
  static constexpr int REM = L / NS;
  static constexpr int R = REM >= E ? E : REM;
  static constexpr int NB = E / R;                       // butterflies per thread
  static constexpr int NTW = NS > 1 ? NB * (R - 1) : 0;  // twiddles per thread
  static constexpr bool LAST = NS * R == L;
};

template <int L, int E, int NS>
struct StageTw {
  float2 w[StagePlan<L, E, NS>::NTW > 0 ? StagePlan<L, E, NS>::NTW : 1];
};

// Loads the twiddles of the stage starting at span NS (from the stage section,
// contiguous across the lanes of a wave).
template <int L, int E, int NS, class TS>
__device__ __forceinline__ void load_stage_tw(StageTw<L, E, NS>& tw, int t, bool active, const TS& ts) {
  using P = StagePlan<L, E, NS>;
  if constexpr (P::NTW > 0) {
    if (!active) return;
#pragma unroll
    for (int b = 0; b < P::NB; ++b) {
      const int k = (t + P::T * b) & (NS - 1);
#pragma unroll
      for (int m = 1; m < P::R; ++m) tw.w[b * (P::R - 1) + m - 1] = ts.template stage<NS, P::R>(k, m);
    }
  }
}

// Stages from span NS onward: radix E while at least E remains, then the
// remainder as the last stage.  `tw` holds this stage's twiddles; the next
// stage's are fetched before the LDS exchange so their latency overlaps it.
// `active` = false skips arithmetic and LDS traffic but keeps the barriers.
template <int L, int E, int NS, bool INV, class TS, class DF>
__device__ __forceinline__ void fft_stages_tw(float2 (&v)[E], float2* lds, int t, bool active,
                                              const StageTw<L, E, NS>& tw, const TS& ts, const DF& df) {
  using P = StagePlan<L, E, NS>;
  constexpr int T = P::T, R = P::R, NB = P::NB;
  // a wave-wide DFT runs on every lane (inactive lanes transform garbage and store nothing)
  constexpr bool kAll = DF::kWave && R == 16;
  if constexpr (L / NS > 1) {
    if (active || kAll) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        float2 x[R];
#pragma unroll
        for (int m = 0; m < R; ++m) x[m] = v[b + m * NB];
        const int j = t + T * b;
        const int k = j & (NS - 1);
        if constexpr (NS > 1) {
#pragma unroll
          for (int m = 1; m < R; ++m) {
            const float2 w = tw.w[b * (R - 1) + m - 1];
            x[m] = INV ? cmulc(x[m], w) : cmul(x[m], w);
          }
        }
        df.template run<R, INV>(x);
        if constexpr (P::LAST) {
#pragma unroll
          for (int m = 0; m < R; ++m) v[b + m * NB] = x[m];
        } else if (active) {
          const int base = (j - k) * R + k;
          if constexpr (NS % 16 == 0 || NS * R <= 16) {
            // base + m NS never crosses a 16-entry group boundary that
            // pad(base) has not already counted (NS R <= 16), or crosses
            // exactly m NS / 16 of them (NS a multiple of 16): the padded
            // index is pad(base) plus a constant per m
            const int pb = lds_pad(base);
#pragma unroll
            for (int m = 0; m < R; ++m) lds[pb + m * NS + (NS % 16 == 0 ? m * NS / 16 : 0)] = x[m];
          } else {
#pragma unroll
            for (int m = 0; m < R; ++m) lds[lds_pad(base + m * NS)] = x[m];
          }
        }
      }
    }
    if constexpr (!P::LAST) {
      StageTw<L, E, NS * R> next;
      if constexpr (!TwFetchLate<TS>::value) load_stage_tw<L, E, NS * R>(next, t, active, ts);
      team_sync<T>();
      if (active) {
        if constexpr (T % 16 == 0) {
          // t < T and T e a multiple of 16: pad(t + T e) = pad(t) + (T + T/16) e
          const int pt = lds_pad(t);
#pragma unroll
          for (int e = 0; e < E; ++e) v[e] = lds[pt + (T + T / 16) * e];
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) v[e] = lds[lds_pad(t + T * e)];
        }
      }
      if constexpr (TwFetchLate<TS>::value) load_stage_tw<L, E, NS * R>(next, t, active, ts);
      if constexpr (T > 64) {
        __syncthreads();
      } else {
        // keep the next stage's LDS writes after these reads (the LDS then
        // serves them in order)
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      }
      fft_stages_tw<L, E, NS * R, INV>(v, lds, t, active, next, ts, df);
    }
  }
}

template <int L, int E, int NS, bool INV, class TS = TwGlobal, class DF = DftFp32>
__device__ __forceinline__ void fft_stages(float2 (&v)[E], float2* lds, int t, bool active, const TS& ts = TS{},
                                           const DF& df = DF{}) {
  StageTw<L, E, NS> tw;
  load_stage_tw<L, E, NS>(tw, t, active, ts);
  fft_stages_tw<L, E, NS, INV>(v, lds, t, active, tw, ts, df);
}

// Full L-point transform of the team's data (cyclic layout in and out).
// Every thread of the work-group must call it when teams span several waves
// (it then contains work-group barriers).
template <int L, int E, bool INV, class DF = DftFp32>
__device__ __forceinline__ void team_fft(float2 (&v)[E], float2* lds, int t, bool active = true,
                                         const DF& df = DF{}) {
  static_assert(L >= E && (L & (L - 1)) == 0, "FFT length");
  static_assert(E == 4 || E == 8 || E == 16, "elements per thread");
  fft_stages<L, E, 1, INV>(v, lds, t, active, TwGlobal{}, df);
}

// Twiddle blocks of one FFT plan (the stages of team_fft from span NS0 on,
// radix E), packed one after another: used to copy a plan's twiddles into LDS.
template <int L, int E, int NS0>
struct PlanTable {
  static constexpr int r_at(int ns) { return L / ns >= E ? E : L / ns; }
  // entries of the twiddle blocks of the stages from NS0 up to (not incl.) NS
  static constexpr int off(int NS) {
    int tot = 0;
    for (int ns = NS0; ns < NS && ns < L; ns *= r_at(ns))
      if (ns > 1) tot += ns * r_at(ns);
    return tot;
  }
  static constexpr int size() { return off(L); }
};

template <int N, int BASE, int NS0>
struct PlanLayout {
  template <int NS, int R>
  static constexpr int off() {
    return BASE + PlanTable<N, 16, NS0>::off(NS);
  }
};

template <int L, int E, int NS0>
__device__ __forceinline__ void copy_plan_twiddles(float2* dst, int tid, int nthreads) {
  using PT = PlanTable<L, E, NS0>;
  int pos = 0;
  for (int ns = NS0; ns < L; ns *= PT::r_at(ns)) {
    const int r = PT::r_at(ns);
    if (ns > 1) {
      const int src = stage_offset(ilog2c(ns), ilog2c(r));
      for (int i = tid; i < ns * r; i += nthreads) dst[pos + i] = g_radar_tw[(unsigned)(src + i)];
      pos += ns * r;
    }
  }
}

}  // namespace radar
