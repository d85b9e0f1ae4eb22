// Host side of libradar: argument validation, workspace carving, the twiddle
// table, and kernel launches behind the C ABI declared in include/radar.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/radar.h"
#include "device_common.hpp"

__device__ float2 g_radar_tw[RADAR_TW_ENTRIES];

#include "k_frame.hpp"
#include "k_range_mx.hpp"
#include "k_range_wide.hpp"
#include "k_peaks.hpp"
#include "k_peaks_only.hpp"
#include "k_refine.hpp"
#include "k_sft.hpp"
#include "k_sft_general.hpp"
#include "k_cnn.hpp"
#include "k_dense.hpp"
#include "k_sim.hpp"

__device__ double2 g_root64_hi[1 << (RADAR_ROOT64_LOG2 - 12)];
__device__ double2 g_root64_lo[1 << 12];

// The workspace of radar_frame_process_noalloc: one array per device, held
// until the process ends.  Host code never uses this name as an address (in
// host code it is a stand-in for the symbol, not device memory): radar_init
// looks up each device's copy with hipGetSymbolAddress and keeps it in
// g_scratch_dev.
static __device__ __align__(256) unsigned char scratch[RADAR_NOALLOC_WS_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_init_mu;
bool g_init_done[kMaxDevices];
void* g_scratch_dev[kMaxDevices];  // device address of `scratch` on each device, set by radar_init

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
int ilog2(int64_t x) {
  int r = 0;
  while ((int64_t(1) << r) < x) ++r;
  return r;
}
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int validate_desc(const radar_frame_desc* d) {
  if (!d) return RADAR_E_ARG;
  const int N = d->n_sub, M = d->n_sym;
  if (N <= 0 || M <= 0 || d->n_pad <= 0 || d->m_pad <= 0) return RADAR_E_ARG;
  if (d->n_pad < N || d->m_pad < M) return RADAR_E_ARG;
  if (d->n_cp < 1 || d->n_cp > N) return RADAR_E_ARG;
  if (d->window < RADAR_WIN_RECT || d->window > RADAR_WIN_HAMMING) return RADAR_E_ARG;
  if (d->zc_mode != RADAR_ZC_NONE && d->zc_mode != RADAR_ZC_DIAG && d->zc_mode != RADAR_ZC_DENSE)
    return RADAR_E_ARG;
  if ((d->flags & ~(RADAR_FLAG_REFINE | RADAR_FLAG_BF16X3 | RADAR_FLAG_FP16X3 | RADAR_FLAG_THRESHOLD |
                    RADAR_FLAG_FP16)) != 0)
    return RADAR_E_ARG;
  if ((d->flags & RADAR_FLAG_THRESHOLD) &&
      !(d->pfa > 0.0f && d->pfa < 1.0f && d->noise_power > 0.0f && d->noise_power <= FLT_MAX))
    return RADAR_E_ARG;
  {
    const int pf = d->flags & (RADAR_FLAG_BF16X3 | RADAR_FLAG_FP16X3 | RADAR_FLAG_FP16);
    if (pf & (pf - 1)) return RADAR_E_ARG;  // at most one precision form
  }
  if (d->ld < N) return RADAR_E_ARG;
  if (reinterpret_cast<uintptr_t>(d->tap_weights) & 3) return RADAR_E_ARG;
  if (!is_pow2(N) || !is_pow2(M) || N < 16 || N > 4096 || M < 16 || M > 4096) return RADAR_E_UNSUPPORTED;
  if (!is_pow2(d->n_pad) || !is_pow2(d->m_pad)) return RADAR_E_UNSUPPORTED;
  if (d->n_pad / N > 8 || d->n_pad > RADAR_TW_LMAX || d->m_pad > RADAR_TW_LMAX) return RADAR_E_UNSUPPORTED;
  if (d->zc_mode != RADAR_ZC_NONE && (d->zc_root % 2) == 0) return RADAR_E_NOT_COPRIME;  // N is a power of two
  if ((d->flags & RADAR_FLAG_REFINE) && (d->m_pad / M > 16 || d->n_pad / N > 16 || M > 1024))
    return RADAR_E_UNSUPPORTED;
  // the matrix-core forms exist for the 4x range-padding kernels
  if ((d->flags & (RADAR_FLAG_BF16X3 | RADAR_FLAG_FP16X3)) && !(d->n_pad == 4 * N && 4 * d->n_cp <= N && N >= 256))
    return RADAR_E_UNSUPPORTED;
  // the single-rounding FP16 form exists for the N = 1024 matrix-core range stage
  if ((d->flags & RADAR_FLAG_FP16) && !(N == 1024 && d->n_pad == 4 * N && 4 * d->n_cp <= N))
    return RADAR_E_UNSUPPORTED;
  return RADAR_OK;
}

// Scratch of the peak search for F frames of m_pad rows (offsets in bytes).
struct PeakWs {
  size_t rowmax, tau, cnt, start, list, cand, total;
};
PeakWs peak_ws_layout(int m_pad, int n_frames, int k, size_t base) {
  PeakWs w;
  const size_t F = (size_t)n_frames;
  w.rowmax = base;
  w.tau = w.rowmax + align256(F * m_pad * sizeof(float));
  w.cnt = w.tau + align256(F * sizeof(float));
  w.start = w.cnt + align256(F * sizeof(int32_t));  // peaks only: first entry of the second listing
  w.list = w.start + align256(F * sizeof(int32_t));
  w.cand = w.list + align256(F * m_pad * sizeof(int32_t));
  w.total = w.cand + align256(F * m_pad * (size_t)k * sizeof(uint64_t));
  return w;
}

struct FrameWs {
  size_t taps, U;
  PeakWs pk;
  size_t inv_sum;  // [F][M] floats with RADAR_FLAG_THRESHOLD (else an empty region)
  size_t H;        // [F][M][N] LS estimate with RADAR_ZC_DENSE at N outside 256 .. 1024 (else empty)
  size_t ring;     // peaks only: the recompute kernel's row rings
  size_t total;
};

bool peaks_only_supported(const radar_frame_desc* d);

// Peaks only: work-groups of the recompute kernel (two per frame up to one
// per CU of the largest part) and the bytes of their row rings (8 wavefronts,
// each 1024/N + 2 rows of 4N floats).
int window_blocks(int n_frames) { return std::min(256, 2 * n_frames); }
size_t window_ring_bytes(int N, int n_frames) {
  return (size_t)window_blocks(n_frames) * 8 * (size_t)(1024 / N + 2) * (size_t)(4 * N) * sizeof(float);
}

FrameWs frame_ws_layout(const radar_frame_desc* d, int n_frames, int k) {
  FrameWs w;
  const size_t F = (size_t)n_frames;
  w.taps = 0;
  w.U = align256(F * d->n_sym * d->n_cp * sizeof(float2));
  w.pk = peak_ws_layout(d->m_pad, n_frames, k, w.U + align256(F * d->m_pad * d->n_cp * sizeof(float2)));
  w.inv_sum = w.pk.total;
  w.H = w.inv_sum + ((d->flags & RADAR_FLAG_THRESHOLD) ? align256(F * d->n_sym * sizeof(float)) : 0);
  // the estimate passes through HBM only where the taps kernel does not
  // take the dense precoding itself
  const bool h_in_hbm = d->zc_mode == RADAR_ZC_DENSE && (d->n_sub < 256 || d->n_sub > 1024);
  w.ring = w.H + (h_in_hbm ? align256(F * d->n_sym * (size_t)d->n_sub * sizeof(float2)) : 0);
  w.total = w.ring;
  // the rings live in the taps region, dead once the Doppler stage has read
  // it, unless the refinement reads the taps later or the region is too small
  if (peaks_only_supported(d)) {
    const size_t ring = window_ring_bytes(d->n_sub, n_frames);
    if ((d->flags & RADAR_FLAG_REFINE) || ring > w.U - w.taps)
      w.total += align256(ring);
    else
      w.ring = w.taps;
  }
  return w;
}

// sum_{n<L} w_n^2 of the periodic windows (full periods of the cosine, L >= 16)
double window_energy(int kind, int L) {
  if (kind == RADAR_WIN_HANN) return 0.375 * L;                  // 1/4 + 1/8
  if (kind == RADAR_WIN_HAMMING) return (0.54 * 0.54 + 0.5 * 0.46 * 0.46) * L;
  return (double)L;
}

// eta = eta_factor * sum_{l,k} 1/|a_{l,k}|^2: -ln(pfa) sigma^2 mean(1/|a|^2)
// sum_l w_l^2 sum_k w_k^2 / (N M), the mean taken as the sum over N M.
float eta_factor_of(const radar_frame_desc* d) {
  const double nm = (double)d->n_sub * (double)d->n_sym;
  return (float)(-std::log((double)d->pfa) * (double)d->noise_power * window_energy(d->window, d->n_sym) *
                 window_energy(d->window, d->n_sub) / (nm * nm));
}

int ensure_init() { return radar_init(); }

// ----------------------------------------------------------- stage timing
struct StageTimer {
  bool on = false;
  int cap = 0;
  int used[RADAR_NUM_STAGES] = {};
  std::vector<hipEvent_t> ev[RADAR_NUM_STAGES];  // 2 per launch
};
StageTimer g_timer;
thread_local bool g_capturing = false;  // launches are being captured into a graph: no event records

// Launch parameters an autotuner may choose per shape (defaults: one
// persistent work-group per CU, the four-phase range kernel where it applies).
struct Tuning {
  int k1_mult = 1;         // persistent taps kernel: work-groups per CU
  int k3_mult = 1;         // persistent range kernel: work-groups per CU
  bool k3_generic = false; // use the one-team-per-row range kernel instead of the four-phase one
  bool k2_half = false;    // Doppler tiles of half the taps (FP32)
  int scan_groups = 32;    // work-groups per frame of the listed-row peak scan
  float ms = 0.0f;         // measured time of one pass of the group with these settings (0: not measured)
};
thread_local Tuning g_tune;
int g_num_cus = 0;  // compute units of the device, set by radar_init

// Records the opening event of a timed stage launch; returns the slot or -1.
int timer_open(int stage, hipStream_t s) {
  if (g_capturing || !g_timer.on || g_timer.used[stage] >= g_timer.cap) return -1;
  const int slot = g_timer.used[stage]++;
  (void)hipEventRecord(g_timer.ev[stage][2 * slot], s);
  return slot;
}
void timer_close(int stage, int slot, hipStream_t s) {
  if (slot >= 0) (void)hipEventRecord(g_timer.ev[stage][2 * slot + 1], s);
}

#define RADAR_HIP_CHECK(expr)                  \
  do {                                         \
    if ((expr) != hipSuccess) return RADAR_E_HIP; \
  } while (0)

// ----------------------------------------------------------------- dispatch
template <int N>
void launch_k1p_n(const radar::K1Args& a, int M, int F, hipStream_t s);
template <int N>
void launch_k1_n(const radar::K1Args& a, int M, int F, hipStream_t s) {
  if constexpr (N >= 256 && N <= 1024) {
    launch_k1p_n<N>(a, M, F, s);
    return;
  }
  constexpr int TEAMS = radar::kBlock / (N / 16);
  dim3 grid((M + TEAMS - 1) / TEAMS, F);
  hipLaunchKernelGGL(radar::k1_taps<N>, grid, dim3(radar::kBlock), 0, s, a);
}
template <int M, int TW, radar::Prec PR>
void launch_k2_tw(const radar::K2Args& a, int n_cp, int F, hipStream_t s) {
  // persistent: as many work-groups as fit on the device at once (a static
  // initialised once, thread-safely, on the first call for this shape)
  static const int per_cu = [] {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, radar::k2_doppler_tiled<M, TW, PR>,
                                                     radar::K2Tile<M, TW>::BLOCK, 0) != hipSuccess ||
        v < 1)
      v = 1;
    return v;
  }();
  const int n_tiles = (n_cp + TW - 1) / TW;
  const int total = n_tiles * a.fm * F;
  int grid = (g_num_cus > 0 ? g_num_cus : 256) * per_cu;
  if (grid > total || !radar::K2Persistent<PR>::value) grid = total;
  hipLaunchKernelGGL((radar::k2_doppler_tiled<M, TW, PR>), dim3(grid), dim3(radar::K2Tile<M, TW>::BLOCK), 0, s, a,
                     n_tiles, total);
}
template <int M, radar::Prec PR>
void launch_k2_m(const radar::K2Args& a, int n_cp, int F, hipStream_t s) {
  // tiles of TW taps: at most 64, at most 1024 threads, padded tile M*(TW+1) <= 17408 entries
  constexpr int T = M / 16;
  constexpr int TW0 = 1024 / T < 64 ? 1024 / T : 64;
  constexpr int TW = M * (TW0 + 1) <= 17408 ? TW0 : 17408 / M - 1;
  // the autotuner's alternative (FP32, M >= 64): tiles of half the taps and
  // about half the LDS (two work-groups per CU where two fit)
  if constexpr (PR == radar::Prec::FP32 && M >= 64 && TW >= 2) {
    if (g_tune.k2_half) {
      launch_k2_tw<M, TW / 2, PR>(a, n_cp, F, s);
      return;
    }
  }
  launch_k2_tw<M, TW, PR>(a, n_cp, F, s);
}
template <int N, int F2>
void launch_k3_nf(const radar::K3Args& a, int m_pad, int F, hipStream_t s) {
  constexpr int TEAMS = radar::kBlock / (N / 16);
  dim3 grid((m_pad + TEAMS - 1) / TEAMS, F);
  hipLaunchKernelGGL((radar::k3_range_power<N, F2>), grid, dim3(radar::kBlock), 0, s, a);
}
template <int N, radar::Prec PR>
void launch_k3x4_n(const radar::K3Args& a, int m_pad, int F, hipStream_t s) {
  using C = radar::K3x4<N>;
  dim3 grid(m_pad / C::ROWS, F);
  hipLaunchKernelGGL((radar::k3_range_power_x4<N, PR>), grid, dim3(C::BLOCK), 0, s, a);
}
template <int N>
void launch_k1p_n(const radar::K1Args& a, int M, int F, hipStream_t s) {
  using C = radar::K1p<N>;
  const int total = (int)((int64_t)F * M / C::ROWS);
  int grid = (g_num_cus > 0 ? g_num_cus : 256) * g_tune.k1_mult;
  if (grid * C::WAVES > total) grid = (total + C::WAVES - 1) / C::WAVES;
  hipLaunchKernelGGL(radar::k1_taps_p<N>, dim3(grid), dim3(C::BLOCK), 0, s, a, total);
}
// the taps stage with the dense precoding folded in (N = 256 .. 1024)
template <int N>
void launch_k1d_n(const radar::K1Args& a, int M, int F, hipStream_t s) {
  using C = radar::K1d<N>;
  const int total = (int)((int64_t)F * M / C::ROWS);
  int grid = (g_num_cus > 0 ? g_num_cus : 256) * g_tune.k1_mult;
  if (grid * C::WAVES > total) grid = (total + C::WAVES - 1) / C::WAVES;
  hipLaunchKernelGGL(radar::k1_taps_dense<N>, dim3(grid), dim3(C::BLOCK), 0, s, a, total);
}
template <int N>
void launch_dense_n(const radar::DenseArgs& a, hipStream_t s) {
  // persistent: as many work-groups as fit on the device at once (a static
  // initialised once, thread-safely, on the first call for this size)
  static const int per_cu = [] {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, radar::k_dense_ls<N>, radar::kDenseThreads, 0) !=
            hipSuccess ||
        v < 1)
      v = 1;
    return v;
  }();
  int grid = (g_num_cus > 0 ? g_num_cus : 256) * per_cu;
  if (grid > a.total) grid = a.total;
  hipLaunchKernelGGL(radar::k_dense_ls<N>, dim3(grid), dim3(radar::kDenseThreads), 0, s, a);
}
template <int N, radar::Prec PR, bool kStore = true>
void launch_k3x4p_n(const radar::K3Args& a, int m_pad, int F, hipStream_t s) {
  using C = radar::K3p<N>;
  const int total = (int)((int64_t)F * m_pad / C::ROWS);
  const int per_wg = C::WAVES;
  int grid = (g_num_cus > 0 ? g_num_cus : 256) * g_tune.k3_mult;
  if (grid * per_wg > total) grid = (total + per_wg - 1) / per_wg;
  if constexpr (kStore) {
    if (a.refs) {
      hipLaunchKernelGGL((radar::k3_range_power_x4p<N, PR, true, true>), dim3(grid), dim3(C::BLOCK), 0, s, a, total);
      return;
    }
  }
  hipLaunchKernelGGL((radar::k3_range_power_x4p<N, PR, kStore, false>), dim3(grid), dim3(C::BLOCK), 0, s, a, total);
}
// the N = 2048 range kernel (FP32): persistent, one work-group per CU (its
// LDS holds one)
void launch_k3x4w(const radar::K3Args& a, int m_pad, int F, hipStream_t s) {
  using C = radar::K3w<2048>;
  const int total = F * m_pad;
  int grid = (g_num_cus > 0 ? g_num_cus : 256) * g_tune.k3_mult;
  if (grid * C::PAIRS > total) grid = (total + C::PAIRS - 1) / C::PAIRS;
  if (a.refs)
    hipLaunchKernelGGL((radar::k3_range_power_x4w<2048, true>), dim3(grid), dim3(C::BLOCK), 0, s, a, total);
  else
    hipLaunchKernelGGL((radar::k3_range_power_x4w<2048, false>), dim3(grid), dim3(C::BLOCK), 0, s, a, total);
}
// the matrix-core range kernel (N = 1024): one persistent work-group per CU
template <radar::Prec PR, bool kStore = true>
void launch_k3mx(const radar::K3Args& a, int m_pad, int F, hipStream_t s) {
  using C = radar::K3Mx<1024>;
  const int total = (int)((int64_t)F * m_pad);
  int grid = (g_num_cus > 0 ? g_num_cus : 256) * g_tune.k3_mult;
  if (grid * C::WAVES > total) grid = (total + C::WAVES - 1) / C::WAVES;
  if constexpr (kStore) {
    if (a.refs) {
      hipLaunchKernelGGL((radar::k3_range_power_mx<1024, PR, true, true>), dim3(grid), dim3(C::BLOCK), 0, s, a,
                         total);
      return;
    }
  }
  hipLaunchKernelGGL((radar::k3_range_power_mx<1024, PR, kStore, false>), dim3(grid), dim3(C::BLOCK), 0, s, a,
                     total);
}
template <int N>
void launch_k3_n(const radar::K3Args& a, int f2, int m_pad, int F, hipStream_t s) {
  switch (f2) {
    case 1: launch_k3_nf<N, 1>(a, m_pad, F, s); break;
    case 2: launch_k3_nf<N, 2>(a, m_pad, F, s); break;
    case 4: launch_k3_nf<N, 4>(a, m_pad, F, s); break;
    default: launch_k3_nf<N, 8>(a, m_pad, F, s); break;
  }
}

#define RADAR_SIZE_SWITCH(n, CALL) \
  switch (n) {                     \
    case 16: CALL(16); break;      \
    case 32: CALL(32); break;      \
    case 64: CALL(64); break;      \
    case 128: CALL(128); break;    \
    case 256: CALL(256); break;    \
    case 512: CALL(512); break;    \
    case 1024: CALL(1024); break;  \
    case 2048: CALL(2048); break;  \
    default: CALL(4096); break;    \
  }

template <radar::Prec PR>
void launch_k3x4_any(const radar::K3Args& a, int N, int m_pad, int F, hipStream_t s) {
  switch (N) {
    case 256: launch_k3x4p_n<256, PR>(a, m_pad, F, s); break;
    case 512: launch_k3x4p_n<512, PR>(a, m_pad, F, s); break;
    case 1024: launch_k3x4p_n<1024, PR>(a, m_pad, F, s); break;
    case 2048:
      if constexpr (PR == radar::Prec::FP32)
        launch_k3x4w(a, m_pad, F, s);
      else
        launch_k3x4_n<2048, PR>(a, m_pad, F, s);
      break;
    default: launch_k3x4_n<4096, PR>(a, m_pad, F, s); break;
  }
}

// P not materialised: the row maxima only (the x4p shapes; the caller checked
// peaks_only_supported)
template <radar::Prec PR>
void launch_k3x4p_rowmax(const radar::K3Args& a, int N, int m_pad, int F, hipStream_t s) {
  switch (N) {
    case 256: launch_k3x4p_n<256, PR, false>(a, m_pad, F, s); break;
    case 512: launch_k3x4p_n<512, PR, false>(a, m_pad, F, s); break;
    default: launch_k3x4p_n<1024, PR, false>(a, m_pad, F, s); break;
  }
}
template <radar::Prec PR>
void launch_rows_window(const radar::K3Args& a, int N, int F, int k, const float* tau, const int32_t* list,
                        const int32_t* cnt, const int32_t* start, uint64_t* cand, float* ring, hipStream_t s) {
  // the range kernel's work-group and LDS, one per CU, each building its
  // tables once and then taking (frame, share) items in turn
  const int blocks = window_blocks(F);
  const int per_frame = std::max(1, blocks / F);
  switch (N) {
    case 256:
      hipLaunchKernelGGL((radar::k_peak_rows_window<256, PR>), dim3(blocks), dim3(radar::K3p<256>::BLOCK), 0, s, a,
                         F, per_frame, k, tau, list, cnt, start, cand, ring);
      break;
    case 512:
      hipLaunchKernelGGL((radar::k_peak_rows_window<512, PR>), dim3(blocks), dim3(radar::K3p<512>::BLOCK), 0, s, a,
                         F, per_frame, k, tau, list, cnt, start, cand, ring);
      break;
    default:
      hipLaunchKernelGGL((radar::k_peak_rows_window<1024, PR>), dim3(blocks), dim3(radar::K3p<1024>::BLOCK), 0, s,
                         a, F, per_frame, k, tau, list, cnt, start, cand, ring);
      break;
  }
}

// Shapes whose periodogram need not be materialised: the range kernel of the
// 4x padding with N_cp <= N/4 and N <= 1024 keeps row maxima without writing
// P, and the peak search recomputes the rows it scans.
bool peaks_only_supported(const radar_frame_desc* d) {
  const int N = d->n_sub;
  return (N == 256 || N == 512 || N == 1024) && d->n_pad == 4 * N && d->n_cp * 4 <= N;
}

// The matrix-core range kernel runs the range stage: N = 1024, N' = 4N,
// 4 N_cp <= N, a matrix-core form, P written (or batch jobs).
bool range_on_mx(const radar_frame_desc* d, bool p_written) {
  const int N = d->n_sub;
  return p_written && N == 1024 && d->n_pad == 4 * N && 4 * d->n_cp <= N &&
         (d->flags & (RADAR_FLAG_BF16X3 | RADAR_FLAG_FP16X3 | RADAR_FLAG_FP16)) != 0;
}

radar::Prec prec_of(const radar_frame_desc* d) {
  if (d->flags & RADAR_FLAG_BF16X3) return radar::Prec::BF16X3;
  if (d->flags & RADAR_FLAG_FP16X3) return radar::Prec::FP16X3;
  if (d->flags & RADAR_FLAG_FP16) return radar::Prec::FP16;
  return radar::Prec::FP32;
}

// Arguments of the range stage (and of the peaks-only row recomputation).
radar::K3Args range_args(const radar_frame_desc* d, const float2* U, float* P, int64_t p_stride, float* rowmax,
                         const radar::FrameRef* refs) {
  radar::K3Args a3{};
  a3.U = U;
  a3.P = P;
  a3.p_stride = p_stride;
  a3.m_pad = d->m_pad;
  a3.n_pad = d->n_pad;
  a3.n_cp = d->n_cp;
  a3.window = d->window;
  a3.scale = (float)(1.0 / ((double)d->n_sub * (double)d->n_sym));
  a3.rowmax = rowmax;
  a3.refs = refs;
  return a3;
}

// K1 -> K2 -> K3 for one batch of frames with a common descriptor.
int enqueue_transforms(const radar_frame_desc* d, int F, const float2* in, const float2* A,
                       int64_t frame_stride, int from_h, float* P, int64_t p_stride, uint32_t* status,
                       const FrameWs& w, char* ws, hipStream_t s, const radar::FrameRef* refs = nullptr) {
  const int N = d->n_sub, M = d->n_sym;
  float2* taps = reinterpret_cast<float2*>(ws + w.taps);
  float2* U = reinterpret_cast<float2*>(ws + w.U);

  float* inv_sum = (d->flags & RADAR_FLAG_THRESHOLD) ? reinterpret_cast<float*>(ws + w.inv_sum) : nullptr;
  radar::K1Args a1{};
  a1.Y = in;
  a1.A = A;
  a1.ld = d->ld;
  a1.frame_stride = frame_stride;
  a1.taps = taps;
  a1.status = status;
  a1.M = M;
  a1.n_cp = d->n_cp;
  // ZC root and shift reduced modulo 2N (diagonal) or 2N^2 (dense: the phases
  // of the length-N^2 sequence)
  const bool dense = d->zc_mode == RADAR_ZC_DENSE;
  const int64_t period = dense ? 2 * (int64_t)N * N : 2 * (int64_t)N;
  const bool zc_on = d->zc_mode != RADAR_ZC_NONE;
  a1.zc_root = zc_on ? (uint32_t)(((d->zc_root % period) + period) % period) : 0u;
  a1.zc_shift = zc_on ? (uint32_t)(((d->zc_shift % period) + period) % period) : 0u;
  a1.window = d->window;
  a1.from_h = from_h;
  a1.inv_n = 1.0f / (float)N;
  a1.refs = refs;
  a1.inv_sum = inv_sum;
  a1.tap_w = d->tap_weights;
  int slot = timer_open(RADAR_STAGE_TAPS, s);
  if (dense && N >= 256 && N <= 1024) {
    // the precoding transform inside the taps kernel: the LS estimate stays on chip
    switch (N) {
      case 256: launch_k1d_n<256>(a1, M, F, s); break;
      case 512: launch_k1d_n<512>(a1, M, F, s); break;
      default: launch_k1d_n<1024>(a1, M, F, s); break;
    }
  } else {
    if (dense) {
      // other sizes: the FP64 precoding and division first, the taps kernel
    // then reads the estimate
      radar::DenseArgs ad{};
      ad.Y = in;
      ad.A = A;
      ad.ld = d->ld;
      ad.frame_stride = frame_stride;
      ad.refs = refs;
      ad.status = status;
      ad.H = reinterpret_cast<float2*>(ws + w.H);
      ad.inv_sum = inv_sum;
      ad.M = M;
      ad.total = F * M;
      ad.zc_root = a1.zc_root;
      ad.zc_shift = a1.zc_shift;
#define KD_CALL(n) launch_dense_n<n>(ad, s)
      RADAR_SIZE_SWITCH(N, KD_CALL)
#undef KD_CALL
      RADAR_HIP_CHECK(hipGetLastError());
      a1.Y = ad.H;
      a1.A = nullptr;
      a1.ld = N;
      a1.frame_stride = (int64_t)M * N;
      a1.from_h = 1;
      a1.refs = nullptr;
      a1.status = nullptr;
      a1.inv_sum = nullptr;
    }
#define K1_CALL(n) launch_k1_n<n>(a1, M, F, s)
    RADAR_SIZE_SWITCH(N, K1_CALL)
#undef K1_CALL
  }
  timer_close(RADAR_STAGE_TAPS, slot, s);
  RADAR_HIP_CHECK(hipGetLastError());

  radar::K2Args a2{};
  a2.taps = taps;
  a2.U = U;
  a2.M = M;
  a2.m_pad = d->m_pad;
  a2.n_cp = d->n_cp;
  a2.fm = d->m_pad / M;
  a2.ph_off = (a2.fm == 2 || a2.fm == 4 || a2.fm == 8) ? radar::phase_offset(ilog2(M), ilog2(a2.fm)) : -1;
  slot = timer_open(RADAR_STAGE_DOPPLER, s);
  const radar::Prec prec = prec_of(d);
  const bool mx = range_on_mx(d, P || refs);
  // with the matrix-core range kernel the Doppler stage stays FP32 (it is
  // bound by memory and latency, and its split form measured slower)
  if (prec == radar::Prec::BF16X3 && !mx) {
#define K2_CALL(m) launch_k2_m<m, radar::Prec::BF16X3>(a2, d->n_cp, F, s)
    RADAR_SIZE_SWITCH(M, K2_CALL)
#undef K2_CALL
  } else if (prec == radar::Prec::FP16X3 && !mx) {
#define K2_CALL(m) launch_k2_m<m, radar::Prec::FP16X3>(a2, d->n_cp, F, s)
    RADAR_SIZE_SWITCH(M, K2_CALL)
#undef K2_CALL
  } else {
#define K2_CALL(m) launch_k2_m<m, radar::Prec::FP32>(a2, d->n_cp, F, s)
    RADAR_SIZE_SWITCH(M, K2_CALL)
#undef K2_CALL
  }
  timer_close(RADAR_STAGE_DOPPLER, slot, s);
  RADAR_HIP_CHECK(hipGetLastError());

  const radar::K3Args a3 = range_args(d, U, P, p_stride, reinterpret_cast<float*>(ws + w.pk.rowmax), refs);
  const int f2 = d->n_pad / N;
  const bool x4 = f2 == 4 && d->n_cp * 4 <= N && N >= 256 && !(g_tune.k3_generic && prec == radar::Prec::FP32);
  slot = timer_open(RADAR_STAGE_RANGE, s);
  if (!P && !refs) {
    // peaks only: row maxima, no P (peaks_only_supported was checked); the
    // FP16 form's from its matrix-core kernel where it has one (N = 1024;
    // elsewhere it runs in FP32)
    if (prec == radar::Prec::FP16 && range_on_mx(d, true))
      launch_k3mx<radar::Prec::FP16, false>(a3, d->m_pad, F, s);
    else if (prec == radar::Prec::BF16X3)
      launch_k3x4p_rowmax<radar::Prec::BF16X3>(a3, N, d->m_pad, F, s);
    else if (prec == radar::Prec::FP16X3)
      launch_k3x4p_rowmax<radar::Prec::FP16X3>(a3, N, d->m_pad, F, s);
    else
      launch_k3x4p_rowmax<radar::Prec::FP32>(a3, N, d->m_pad, F, s);
  } else if (mx) {
    if (prec == radar::Prec::BF16X3)
      launch_k3mx<radar::Prec::BF16X3>(a3, d->m_pad, F, s);
    else if (prec == radar::Prec::FP16X3)
      launch_k3mx<radar::Prec::FP16X3>(a3, d->m_pad, F, s);
    else
      launch_k3mx<radar::Prec::FP16>(a3, d->m_pad, F, s);
  } else if (x4) {
    if (prec == radar::Prec::BF16X3)
      launch_k3x4_any<radar::Prec::BF16X3>(a3, N, d->m_pad, F, s);
    else if (prec == radar::Prec::FP16X3)
      launch_k3x4_any<radar::Prec::FP16X3>(a3, N, d->m_pad, F, s);
    else
      launch_k3x4_any<radar::Prec::FP32>(a3, N, d->m_pad, F, s);
  } else {
#define K3_CALL(n) launch_k3_n<n>(a3, f2, d->m_pad, F, s)
    RADAR_SIZE_SWITCH(N, K3_CALL)
#undef K3_CALL
  }
  timer_close(RADAR_STAGE_RANGE, slot, s);
  RADAR_HIP_CHECK(hipGetLastError());
  if (!x4 && (P || refs)) {
    hipLaunchKernelGGL(radar::k_row_max, dim3(d->m_pad, F), dim3(256), 0, s, P, p_stride, d->m_pad, d->n_pad,
                       a3.rowmax, refs);
    RADAR_HIP_CHECK(hipGetLastError());
  }
  return RADAR_OK;
}

// Sub-cell refinement of the k peaks of every frame from the DFT-CE taps.
int enqueue_refine(const radar_frame_desc* d, int F, int k, const float2* taps, radar_peak* peaks,
                   int32_t* n_peaks, const radar::FrameRef* refs, hipStream_t s) {
  radar::K7Args a7{};
  a7.taps = taps;
  a7.peaks = peaks;
  a7.n_peaks = n_peaks;
  a7.k = k;
  a7.M = d->n_sym;
  a7.N = d->n_sub;
  a7.n_cp = d->n_cp;
  a7.m_pad = d->m_pad;
  a7.n_pad = d->n_pad;
  a7.window = d->window;
  a7.refs = refs;
  const int slot = timer_open(RADAR_STAGE_REFINE, s);
  hipLaunchKernelGGL(radar::k7_refine, dim3(k, F), dim3(radar::kRefineThreads), 0, s, a7);
  timer_close(RADAR_STAGE_REFINE, slot, s);
  RADAR_HIP_CHECK(hipGetLastError());
  return RADAR_OK;
}

// Peak search from P and its row maxima (already in the workspace).
// With inv_sum (threshold detection) the merge keeps only peaks at or above eta.
// Peaks only: the relative error bound of the range stage's row maxima
// against the rows the peak search recomputes.  The FP32 and split forms
// recompute with their own row code, compiled into another kernel (a few
// ulps); the FP16 form's maxima come from its matrix-core kernel and the rows
// are recomputed in FP32, so the bound is that form's error with a wide
// margin (its rows are scaled one by one; the largest relative difference
// measured at a peak is 1.3e-3).
float peaks_only_slack(const radar_frame_desc* d) {
  return (d->flags & RADAR_FLAG_FP16) && range_on_mx(d, true) ? 1.0f / 32.0f : 1.0f / 65536.0f;
}
// RADAR_PEAKS_ONLY_FIRST_ROWS = R (1..64, a diagnostic): the first listing
// keeps only the R rows with the largest maxima, so that the second listing
// finds the rest (tests use it to exercise that listing).
int peaks_only_first_rows() {
  const char* e = std::getenv("RADAR_PEAKS_ONLY_FIRST_ROWS");
  if (!e) return 0;
  const int r = std::atoi(e);
  return r < 1 ? 0 : (r > 64 ? 64 : r);
}

// With P null (peaks only, frame_process) the listed rows are recomputed from
// the Doppler-tap rows U by the range kernel's row code (`d` and `U` given).
int enqueue_peaks(const float* P, int64_t p_stride, int m_pad, int n_pad, int F, int k, const PeakWs& w, char* ws,
                  radar_peak* peaks, int32_t* n_peaks, hipStream_t s, const radar::FrameRef* refs = nullptr,
                  const float* inv_sum = nullptr, int M = 0, float eta_factor = 0.0f,
                  const radar_frame_desc* d = nullptr, const float2* U = nullptr, float* ring = nullptr) {
  float* rowmax = reinterpret_cast<float*>(ws + w.rowmax);
  float* tau = reinterpret_cast<float*>(ws + w.tau);
  int32_t* cnt = reinterpret_cast<int32_t*>(ws + w.cnt);
  int32_t* list = reinterpret_cast<int32_t*>(ws + w.list);
  uint64_t* cand = reinterpret_cast<uint64_t*>(ws + w.cand);
  const int slot = timer_open(RADAR_STAGE_PEAKS, s);
  const bool recompute = !P && !refs;
  if (recompute && (!d || !U || !ring)) return RADAR_E_ARG;
  // peaks only: the rows scanned are recomputed in FP32 or the split form
  // by another kernel than the one whose row maxima set tau.  Those maxima
  // differ from the recomputed ones by a few ulps, or, from the FP16
  // matrix-core range kernel, by that form's error: at most peaks_only_slack
  // relative.
  const float slack = recompute ? peaks_only_slack(d) : 0.0f;
  const int first_rows = recompute ? peaks_only_first_rows() : 0;
  hipLaunchKernelGGL(radar::k_peak_threshold, dim3(F), dim3(256), 2 * m_pad * sizeof(uint32_t), s, rowmax, m_pad, k,
                     tau, list, cnt, slack, first_rows);
  RADAR_HIP_CHECK(hipGetLastError());
  if (recompute) {
    const radar::K3Args a3 = range_args(d, U, nullptr, 0, rowmax, nullptr);
    const radar::Prec prec = prec_of(d);
    int32_t* start = reinterpret_cast<int32_t*>(ws + w.start);
    for (int pass = 0; pass < 2; ++pass) {
      const int32_t* st = nullptr;
      if (pass == 1) {
        // the second listing: whatever rows the first one's k-th candidate
        // shows can still hold a top-k peak
        hipLaunchKernelGGL(radar::k_peak_second_listing, dim3(F), dim3(256),
                           ((m_pad + 31) / 32) * sizeof(uint32_t), s, rowmax, m_pad, k, cand, list, cnt, start,
                           slack);
        RADAR_HIP_CHECK(hipGetLastError());
        st = start;
      }
      if (prec == radar::Prec::BF16X3)
        launch_rows_window<radar::Prec::BF16X3>(a3, d->n_sub, F, k, tau, list, cnt, st, cand, ring, s);
      else if (prec == radar::Prec::FP16X3)
        launch_rows_window<radar::Prec::FP16X3>(a3, d->n_sub, F, k, tau, list, cnt, st, cand, ring, s);
      else  // FP32, and the FP16 form's rows again in FP32
        launch_rows_window<radar::Prec::FP32>(a3, d->n_sub, F, k, tau, list, cnt, st, cand, ring, s);
      RADAR_HIP_CHECK(hipGetLastError());
    }
  } else {
    const int groups = m_pad < g_tune.scan_groups ? m_pad : g_tune.scan_groups;
    hipLaunchKernelGGL(radar::k_peak_rows_listed, dim3(groups, F), dim3(256), n_pad * sizeof(uint32_t), s, P,
                       p_stride, m_pad, n_pad, k, tau, list, cnt, cand, refs);
  }
  RADAR_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(radar::k_peak_merge, dim3(F), dim3(256), 0, s, cand, cnt, m_pad, n_pad, k, peaks, n_peaks,
                     refs, inv_sum, M, eta_factor);
  RADAR_HIP_CHECK(hipGetLastError());
  timer_close(RADAR_STAGE_PEAKS, slot, s);
  return RADAR_OK;
}

// ------------------------------------------------------------------ FPS-SFT
struct SftPlan {
  int N, M, Q, n_dirs;
  int dir_a[radar::kSftMaxDirs], dir_b[radar::kSftMaxDirs];
  // Q not a power of two: Q = P R, P a power of two, R odd (the prime-factor path)
  bool general = false;
  int P = 0, R = 1, r_inv = 0, p_inv = 0, gcd_nm = 1;
};

int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a < 0 ? -a : a;
}
// x^-1 mod m (gcd(x, m) = 1, m >= 1) by the extended Euclidean algorithm
int64_t inv_mod(int64_t x, int64_t m) {
  if (m == 1) return 0;
  int64_t r0 = m, r1 = ((x % m) + m) % m, s0 = 0, s1 = 1;
  while (r1) {
    const int64_t q = r0 / r1;
    int64_t t = r0 - q * r1;
    r0 = r1;
    r1 = t;
    t = s0 - q * s1;
    s0 = s1;
    s1 = t;
  }
  return ((s0 % m) + m) % m;
}

int validate_sft(const radar_frame_desc* d, const radar_sft_desc* sd, SftPlan* plan) {
  if (!d || !sd) return RADAR_E_ARG;
  const int N = d->n_sub, M = d->n_sym;
  if (N <= 0 || M <= 0 || d->ld < N || d->flags != 0 || sd->flags != 0) return RADAR_E_ARG;
  if (d->zc_mode != RADAR_ZC_NONE && d->zc_mode != RADAR_ZC_DIAG && d->zc_mode != RADAR_ZC_DENSE)
    return RADAR_E_ARG;
  // the slices gather single elements; dense precoding mixes whole symbols
  if (d->zc_mode == RADAR_ZC_DENSE) return RADAR_E_UNSUPPORTED;
  if (d->tap_weights) return RADAR_E_ARG;  // no DFT-CE taps on this path
  if (sd->n_dirs < 1 || sd->n_dirs > radar::kSftMaxDirs) return RADAR_E_ARG;
  if (sd->k < 1 || sd->k > radar::kSftMaxK) return RADAR_E_ARG;
  if (!(sd->pfa > 0.0f && sd->pfa < 1.0f) || !(sd->tol > 0.0f && sd->tol <= 1.0f)) return RADAR_E_ARG;
  if (N < 16 || N > 4096 || M < 16 || M > 4096) return RADAR_E_UNSUPPORTED;
  if (d->zc_mode == RADAR_ZC_DIAG && gcd64(d->zc_root, N) != 1) return RADAR_E_NOT_COPRIME;
  plan->N = N;
  plan->M = M;
  const int64_t g = gcd64(N, M);
  const int64_t Q = (int64_t)N / g * M;  // lcm(N, M)
  if (is_pow2(Q)) {
    plan->Q = (int)Q;
  } else {
    // the prime-factor path: Q = P R, P = the power of two in Q, R odd
    const int64_t P = Q & -Q, R = Q / P;
    if (Q > radar::kSftGMaxQ || P < 16 || R > radar::kSftGMaxR) return RADAR_E_UNSUPPORTED;
    plan->Q = (int)Q;
    plan->general = true;
    plan->P = (int)P;
    plan->R = (int)R;
    plan->r_inv = (int)inv_mod(R, P);
    plan->p_inv = (int)inv_mod(P, R);
    plan->gcd_nm = (int)g;
  }
  plan->n_dirs = sd->n_dirs;
  for (int i = 0; i < sd->n_dirs; ++i) {
    // alpha enters only through alpha t mod N and alpha k1 Q/N mod Q: reduce mod N (beta mod M)
    const int a = (int)(((int64_t)sd->dirs[i][0] % N + N) % N);
    const int b = (int)(((int64_t)sd->dirs[i][1] % M + M) % M);
    if (a == 0 && b == 0) return RADAR_E_ARG;
    plan->dir_a[i] = a;
    plan->dir_b[i] = b;
  }
  return RADAR_OK;
}

size_t sft_spectra_bytes(const SftPlan& p, int n_frames) {
  return align256((size_t)n_frames * p.n_dirs * 3 * p.Q * sizeof(float2));
}
// the prime-factor path's workspace: the spectra (unless the caller takes
// them), pass 1's output of the same size, conj(z_k) and W_R^x
struct SftGeneralWs {
  size_t S, Z, zc, wr, total;
};
SftGeneralWs sft_general_ws(const SftPlan& p, int n_frames) {
  SftGeneralWs w;
  w.S = 0;
  w.Z = sft_spectra_bytes(p, n_frames);
  w.zc = w.Z + sft_spectra_bytes(p, n_frames);
  w.wr = w.zc + align256((size_t)p.N * sizeof(float2));
  w.total = w.wr + align256((size_t)p.R * sizeof(float2));
  return w;
}

template <int Q>
int launch_sft_q(const radar::K5Args& a5, const radar::K6Args& a6, int F, hipStream_t s);

template <int P>
void launch_sft_pass1(const radar::K5gArgs& g, hipStream_t s) {
  using C = radar::K5Shape<P>;
  const int teams = g.total * g.R;
  hipLaunchKernelGGL(radar::k5g_sft_pass1<P>, dim3((teams + C::TEAMS - 1) / C::TEAMS), dim3(C::BLOCK), 0, s, g);
}

// the prime-factor path: tables, the P-point pass, the R-point pass, the decode
int launch_sft_general(const radar::K5gArgs& g, const radar::K6gArgs& g6, int64_t root, int64_t shift, int F,
                       hipStream_t s) {
  int slot = timer_open(RADAR_STAGE_SFT_SLICES, s);
  const int nt = g.N > g.R ? g.N : g.R;
  hipLaunchKernelGGL(radar::k_sft_tables, dim3((nt + 255) / 256), dim3(256), 0, s, g.N, root, shift, g.R,
                     const_cast<float2*>(g.zc), const_cast<float2*>(g.wr));
  switch (g.P) {
    case 16: launch_sft_pass1<16>(g, s); break;
    case 32: launch_sft_pass1<32>(g, s); break;
    case 64: launch_sft_pass1<64>(g, s); break;
    case 128: launch_sft_pass1<128>(g, s); break;
    case 256: launch_sft_pass1<256>(g, s); break;
    case 512: launch_sft_pass1<512>(g, s); break;
    case 1024: launch_sft_pass1<1024>(g, s); break;
    case 2048: launch_sft_pass1<2048>(g, s); break;
    default: launch_sft_pass1<4096>(g, s); break;
  }
  const int64_t outs = (int64_t)g.total * g.Q;
  hipLaunchKernelGGL(radar::k5g_sft_pass2, dim3((unsigned)((outs + 255) / 256)), dim3(256), 0, s, g);
  timer_close(RADAR_STAGE_SFT_SLICES, slot, s);
  RADAR_HIP_CHECK(hipGetLastError());
  slot = timer_open(RADAR_STAGE_SFT_DECODE, s);
  hipLaunchKernelGGL(radar::k6g_sft_decode, dim3(F), dim3(radar::kSftDecodeThreads), 0, s, g6);
  timer_close(RADAR_STAGE_SFT_DECODE, slot, s);
  RADAR_HIP_CHECK(hipGetLastError());
  return RADAR_OK;
}

template <int Q>
int launch_sft_q(const radar::K5Args& a5, const radar::K6Args& a6, int F, hipStream_t s) {
  using C = radar::K5Shape<Q>;
  int slot = timer_open(RADAR_STAGE_SFT_SLICES, s);
  hipLaunchKernelGGL(radar::k5_sft_slices<Q>, dim3((a5.total + C::TEAMS - 1) / C::TEAMS), dim3(C::BLOCK), 0, s, a5);
  timer_close(RADAR_STAGE_SFT_SLICES, slot, s);
  RADAR_HIP_CHECK(hipGetLastError());
  slot = timer_open(RADAR_STAGE_SFT_DECODE, s);
  hipLaunchKernelGGL(radar::k6_sft_decode<Q>, dim3(F), dim3(radar::kSftDecodeThreads), 0, s, a6);
  timer_close(RADAR_STAGE_SFT_DECODE, slot, s);
  RADAR_HIP_CHECK(hipGetLastError());
  return RADAR_OK;
}

// ------------------------------------------------------------------- CNN
struct CnnWs {
  size_t wb, a1, a2, a3, a4, z5, out, dout, dz5, dz4, dz3, dz2, dz1, part, grad, total;
};

CnnWs cnn_ws_layout(int B, bool train) {
  CnnWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t b = (size_t)B;
  w.wb = take(3 * 9216 * sizeof(__bf16));
  if (!train) {  // inference runs fused: every activation stays in LDS
    w.total = off;
    return w;
  }
  w.a1 = take(b * 32768 * sizeof(__bf16));
  w.a2 = take(b * 8192 * sizeof(__bf16));
  w.a3 = take(b * 8192 * sizeof(__bf16));
  w.a4 = take(b * 2048 * sizeof(__bf16));
  w.z5 = take(b * 10 * sizeof(float));
  w.out = take(b * 2 * sizeof(float));
  w.dout = take(b * 2 * sizeof(float));
  w.dz5 = take(b * 10 * sizeof(float));
  w.dz4 = take(b * 2048 * sizeof(float));
  w.dz3 = take(b * 8192 * sizeof(float));
  w.dz2 = take(b * 8192 * sizeof(float));
  w.dz1 = take(b * 32768 * sizeof(float));
  w.part = take(b * 9248 * sizeof(float));
  w.grad = take(radar::kCnnParams * sizeof(float));
  w.total = off;
  return w;
}

template <int S>
size_t wgrad_lds(int H, int W) {
  return (size_t)(H / S) * (W / S) * 32 * sizeof(float) + (size_t)(H + 2) * (W + 2) * 32 * sizeof(__bf16);
}

std::mutex g_cnn_mu;
int cnn_attrs_done = 0;
int cnn_setup() {
  std::lock_guard<std::mutex> lock(g_cnn_mu);
  if (cnn_attrs_done) return RADAR_OK;
  const int need = (int)wgrad_lds<2>(32, 32);  // the largest weight-gradient tile (conv2)
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(radar::k_conv_wgrad<2>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, need) != hipSuccess ||
      hipFuncSetAttribute(reinterpret_cast<const void*>(radar::k_cnn_fused),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)radar::FusedLds::BYTES) != hipSuccess)
    return RADAR_E_HIP;
  cnn_attrs_done = 1;
  return RADAR_OK;
}

// Inference: the whole network per patch in one persistent kernel.
int cnn_forward_fused(const float* theta, const float* x, int B, const CnnWs& w, char* ws, float* out,
                      hipStream_t s) {
  __bf16* wb = reinterpret_cast<__bf16*>(ws + w.wb);
  hipLaunchKernelGGL(radar::k_cnn_weights_bf16, dim3((3 * 9216 + 255) / 256), dim3(256), 0, s, theta, wb);
  const int grid = std::min(B, g_num_cus > 0 ? g_num_cus : 256);
  hipLaunchKernelGGL(radar::k_cnn_fused, dim3(grid), dim3(radar::kFusedThreads), radar::FusedLds::BYTES, s, x, theta,
                     wb, B, out);
  RADAR_HIP_CHECK(hipGetLastError());
  return RADAR_OK;
}

// The layer-by-layer forward of training (keeps every activation for the backward pass).
int cnn_forward(const float* theta, const float* x, int B, const CnnWs& w, char* ws, float* out, hipStream_t s) {
  __bf16* wb = reinterpret_cast<__bf16*>(ws + w.wb);
  __bf16* a1 = reinterpret_cast<__bf16*>(ws + w.a1);
  __bf16* a2 = reinterpret_cast<__bf16*>(ws + w.a2);
  __bf16* a3 = reinterpret_cast<__bf16*>(ws + w.a3);
  __bf16* a4 = reinterpret_cast<__bf16*>(ws + w.a4);
  float* z5 = reinterpret_cast<float*>(ws + w.z5);
  hipLaunchKernelGGL(radar::k_cnn_weights_bf16, dim3((3 * 9216 + 255) / 256), dim3(256), 0, s, theta, wb);
  hipLaunchKernelGGL(radar::k_conv1_fwd, dim3(B * 4), dim3(256), 0, s, x, theta, a1, B);
  hipLaunchKernelGGL((radar::k_conv_mfma<2, 0>), dim3((B * 8 + 3) / 4), dim3(256), 0, s, a1, wb,
                     theta + radar::kOffConv2B, nullptr, a2, B, 32, 32);
  hipLaunchKernelGGL((radar::k_conv_mfma<1, 0>), dim3((B * 8 + 3) / 4), dim3(256), 0, s, a2, wb + 9216,
                     theta + radar::kOffConv3B, nullptr, a3, B, 16, 16);
  hipLaunchKernelGGL((radar::k_conv_mfma<2, 0>), dim3((B * 2 + 3) / 4), dim3(256), 0, s, a3, wb + 2 * 9216,
                     theta + radar::kOffConv4B, nullptr, a4, B, 16, 16);
  hipLaunchKernelGGL(radar::k_fc_fwd, dim3(B), dim3(256), 0, s, a4, theta, z5, out);
  RADAR_HIP_CHECK(hipGetLastError());
  return RADAR_OK;
}

int cnn_gradient(const float* theta, const float* x, const float* labels, int B, const CnnWs& w, char* ws,
                 float* grad, float* loss, hipStream_t s) {
  float* out = reinterpret_cast<float*>(ws + w.out);
  int rc = cnn_forward(theta, x, B, w, ws, out, s);
  if (rc != RADAR_OK) return rc;
  const __bf16* wb = reinterpret_cast<const __bf16*>(ws + w.wb);
  const __bf16* a1 = reinterpret_cast<const __bf16*>(ws + w.a1);
  const __bf16* a2 = reinterpret_cast<const __bf16*>(ws + w.a2);
  const __bf16* a3 = reinterpret_cast<const __bf16*>(ws + w.a3);
  const __bf16* a4 = reinterpret_cast<const __bf16*>(ws + w.a4);
  const float* z5 = reinterpret_cast<const float*>(ws + w.z5);
  float* dout = reinterpret_cast<float*>(ws + w.dout);
  float* dz5 = reinterpret_cast<float*>(ws + w.dz5);
  float* dz4 = reinterpret_cast<float*>(ws + w.dz4);
  float* dz3 = reinterpret_cast<float*>(ws + w.dz3);
  float* dz2 = reinterpret_cast<float*>(ws + w.dz2);
  float* dz1 = reinterpret_cast<float*>(ws + w.dz1);
  float* part = reinterpret_cast<float*>(ws + w.part);
  hipLaunchKernelGGL(radar::k_mse, dim3(1), dim3(256), 0, s, out, labels, B, dout, loss);
  hipLaunchKernelGGL(radar::k_fc2_bwd, dim3(1), dim3(256), 0, s, dout, z5, theta, B, dz5, grad);
  hipLaunchKernelGGL(radar::k_fc1_wgrad, dim3((20490 + 255) / 256), dim3(256), 0, s, a4, dz5, B, grad);
  hipLaunchKernelGGL(radar::k_fc1_dgrad, dim3(B * 8), dim3(256), 0, s, a4, dz5, theta, B, dz4);
  // conv4 (16x16 -> 8x8)
  hipLaunchKernelGGL((radar::k_conv_wgrad<2>), dim3(B), dim3(256), wgrad_lds<2>(16, 16), s, a3, dz4, part, 16, 16);
  hipLaunchKernelGGL(radar::k_sum_partials, dim3((9248 + 255) / 256), dim3(256), 0, s, part, B, 9248, grad,
                     radar::kOffConv4W);
  hipLaunchKernelGGL((radar::k_conv_mfma<2, 1>), dim3((B * 8 + 3) / 4), dim3(256), 0, s, dz4, wb + 2 * 9216,
                     nullptr, a3, dz3, B, 16, 16);
  // conv3 (16x16 -> 16x16)
  hipLaunchKernelGGL((radar::k_conv_wgrad<1>), dim3(B), dim3(256), wgrad_lds<1>(16, 16), s, a2, dz3, part, 16, 16);
  hipLaunchKernelGGL(radar::k_sum_partials, dim3((9248 + 255) / 256), dim3(256), 0, s, part, B, 9248, grad,
                     radar::kOffConv3W);
  hipLaunchKernelGGL((radar::k_conv_mfma<1, 1>), dim3((B * 8 + 3) / 4), dim3(256), 0, s, dz3, wb + 9216, nullptr,
                     a2, dz2, B, 16, 16);
  // conv2 (32x32 -> 16x16)
  hipLaunchKernelGGL((radar::k_conv_wgrad<2>), dim3(B), dim3(256), wgrad_lds<2>(32, 32), s, a1, dz2, part, 32, 32);
  hipLaunchKernelGGL(radar::k_sum_partials, dim3((9248 + 255) / 256), dim3(256), 0, s, part, B, 9248, grad,
                     radar::kOffConv2W);
  hipLaunchKernelGGL((radar::k_conv_mfma<2, 1>), dim3((B * 32 + 3) / 4), dim3(256), 0, s, dz2, wb, nullptr, a1,
                     dz1, B, 32, 32);
  // conv1
  hipLaunchKernelGGL(radar::k_conv1_wgrad, dim3(B), dim3(256), 0, s, x, dz1, part);
  hipLaunchKernelGGL(radar::k_sum_partials, dim3((320 + 255) / 256), dim3(256), 0, s, part, B, 320, grad,
                     radar::kOffConv1W);
  RADAR_HIP_CHECK(hipGetLastError());
  return RADAR_OK;
}

int cnn_adam(float* theta, const float* grad, float* m, float* v, int step, float lr, hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, step)));
  hipLaunchKernelGGL(radar::k_adam, dim3((radar::kCnnParams + 255) / 256), dim3(256), 0, s, theta, grad, m, v,
                     radar::kCnnParams, lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1,
                     c2);
  RADAR_HIP_CHECK(hipGetLastError());
  return RADAR_OK;
}

// ------------------------------------------------------ uneven batches
struct BatchGroup {
  radar_frame_desc d;
  int k = 0;
  std::vector<int> jobs;
  size_t refs_off = 0;     // FrameRef table in the workspace
  size_t ws_off = 0;  // this group's workspace region (groups may run concurrently)
  double work = 0.0;       // algorithmic bytes, for balancing concurrent branches
  Tuning tune;
};

bool same_group(const radar_frame_desc& a, int ka, const radar_frame_desc& b, int kb) {
  return ka == kb && a.n_sub == b.n_sub && a.n_sym == b.n_sym && a.n_pad == b.n_pad && a.m_pad == b.m_pad &&
         a.n_cp == b.n_cp && a.zc_mode == b.zc_mode && a.zc_root == b.zc_root && a.zc_shift == b.zc_shift &&
         a.window == b.window && a.flags == b.flags && a.ld == b.ld && a.tap_weights == b.tap_weights;
}

int validate_job(const radar_frame_job& j) {
  const int rc = validate_desc(&j.d);
  if (rc != RADAR_OK) return rc;
  if (!j.Y || !j.A || !j.P || !j.peaks || !j.n_peaks || !j.status) return RADAR_E_ARG;
  if (reinterpret_cast<uintptr_t>(j.P) & 15) return RADAR_E_ARG;
  if (j.k < 1 || j.k > 64) return RADAR_E_ARG;
  return RADAR_OK;
}

// groups in order of first appearance; fills the table and workspace offsets and
// returns the workspace size
size_t plan_groups(const radar_frame_job* jobs, int n, std::vector<BatchGroup>& groups) {
  groups.clear();
  for (int i = 0; i < n; ++i) {
    auto it = std::find_if(groups.begin(), groups.end(),
                           [&](const BatchGroup& g) { return same_group(g.d, g.k, jobs[i].d, jobs[i].k); });
    if (it == groups.end()) {
      BatchGroup g;
      g.d = jobs[i].d;
      g.k = jobs[i].k;
      groups.push_back(g);
      it = groups.end() - 1;
    }
    it->jobs.push_back(i);
  }
  size_t off = 0;
  for (auto& g : groups) {
    g.refs_off = off;
    off += align256(g.jobs.size() * sizeof(radar::FrameRef));
  }
  for (auto& g : groups) {
    g.ws_off = off;
    off += frame_ws_layout(&g.d, (int)g.jobs.size(), g.k).total;
    g.work = (double)g.jobs.size() * (16.0 * g.d.n_sub * g.d.n_sym + 4.0 * g.d.n_pad * g.d.m_pad);
  }
  return off;
}

constexpr int kBatchBranches = 4;  // concurrent branches of a captured batch

}  // namespace

struct radar_batch {
  std::vector<BatchGroup> groups;
  char* ws = nullptr;
  int flags = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int enqueue_group(const radar_batch& b, const BatchGroup& g, hipStream_t s) {
  const int F = (int)g.jobs.size();
  const auto* refs = reinterpret_cast<const radar::FrameRef*>(b.ws + g.refs_off);
  char* gws = b.ws + g.ws_off;
  const FrameWs w = frame_ws_layout(&g.d, F, g.k);
  const Tuning saved = g_tune;
  g_tune = g.tune;
  hipLaunchKernelGGL(radar::k0_clear, dim3((F + 255) / 256), dim3(256), 0, s, nullptr, nullptr, F, refs);
  int rc = hipGetLastError() == hipSuccess ? RADAR_OK : RADAR_E_HIP;
  if (rc == RADAR_OK)
    rc = enqueue_transforms(&g.d, F, nullptr, nullptr, 0, 0, nullptr, 0, nullptr, w, gws, s, refs);
  const float* inv_sum =
      (g.d.flags & RADAR_FLAG_THRESHOLD) ? reinterpret_cast<const float*>(gws + w.inv_sum) : nullptr;
  if (rc == RADAR_OK)
    rc = enqueue_peaks(nullptr, 0, g.d.m_pad, g.d.n_pad, F, g.k, w.pk, gws, nullptr, nullptr, s, refs, inv_sum,
                       g.d.n_sym);
  if (rc == RADAR_OK && (g.d.flags & RADAR_FLAG_REFINE))
    rc = enqueue_refine(&g.d, F, g.k, reinterpret_cast<const float2*>(gws + w.taps), nullptr, nullptr, refs, s);
  g_tune = saved;
  return rc;
}

// Autotuner: candidate launch plans of one group, timed on the jobs' data.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int, int, int, int, int, bool, int>, Tuning> g_tune_cache;

int tune_group(radar_batch& b, BatchGroup& g, hipStream_t s) {
  const radar_frame_desc& d = g.d;
  const int F = (int)g.jobs.size();
  // everything that changes the work: the shape, the flags (precision form,
  // refinement, threshold), the precoding (the dense reading adds an FP64
  // stage), tap weights and the window
  const auto key = std::make_tuple(d.n_sub, d.n_sym, d.n_pad, d.m_pad, d.n_cp, d.flags, g.k, F, d.zc_mode,
                                   d.tap_weights != nullptr, d.window);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      g.tune = it->second;
      return RADAR_OK;
    }
  }
  const int N = d.n_sub;
  const bool persistent_k1 = N >= 256 && N <= 1024;
  const bool x4 = d.n_pad == 4 * N && 4 * d.n_cp <= N && N >= 256;
  const bool fp32 = !(d.flags & (RADAR_FLAG_BF16X3 | RADAR_FLAG_FP16X3 | RADAR_FLAG_FP16));
  const bool x4p = x4 && (N <= 1024 || (N == 2048 && fp32));  // a persistent range kernel
  // One dimension at a time, each candidate a change of the best plan so far
  // (every plan is timed, a single one too: the time balances the concurrent
  // branches of the captured batch): work-groups per CU of the persistent
  // taps and range kernels; the range kernel's FFT plan (four N-point phase
  // transforms, or one N'-point transform per row); the Doppler tile width;
  // the peak scan's work-groups per frame.
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return RADAR_E_HIP;
  const auto time_plan = [&](const Tuning& t, float& ms) -> int {
    g.tune = t;
    int rc = enqueue_group(b, g, s);  // warm-up
    if (rc != RADAR_OK) return rc;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < 3 && rc == RADAR_OK; ++r) rc = enqueue_group(b, g, s);
    (void)hipEventRecord(e1, s);
    if (rc != RADAR_OK || hipEventSynchronize(e1) != hipSuccess) return RADAR_E_HIP;
    ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= 3.0f;
    return RADAR_OK;
  };
  Tuning best;
  int rc = time_plan(best, best.ms);
  std::vector<Tuning> alts;
  if (persistent_k1 || x4p) {
    Tuning t;
    t.k1_mult = persistent_k1 ? 2 : 1;
    t.k3_mult = x4p ? 2 : 1;
    alts.push_back(t);
  }
  if (x4 && fp32) {
    Tuning t;
    t.k3_generic = true;
    alts.push_back(t);
  }
  if (fp32 && d.n_sym >= 64) {
    Tuning t;
    t.k2_half = true;
    alts.push_back(t);
  }
  if (d.m_pad > 32) {
    Tuning t;
    t.scan_groups = 128;
    alts.push_back(t);
  }
  for (const Tuning& alt : alts) {
    if (rc != RADAR_OK) break;
    // apply this candidate's changed dimension to the best plan so far
    Tuning t = best;
    if (alt.k1_mult != 1 || alt.k3_mult != 1) {
      t.k1_mult = alt.k1_mult;
      t.k3_mult = alt.k3_mult;
    }
    if (alt.k3_generic) t.k3_generic = true;
    if (alt.k2_half) t.k2_half = true;
    if (alt.scan_groups != 32) t.scan_groups = alt.scan_groups;
    rc = time_plan(t, t.ms);
    if (rc == RADAR_OK && t.ms < best.ms) best = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != RADAR_OK) return rc;
  g.tune = best;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache[key] = g.tune;
  return RADAR_OK;
}

}  // namespace

extern "C" {

int radar_version(void) { return 100; }

const char* radar_status_string(int code) {
  switch (code) {
    case RADAR_OK: return "ok";
    case RADAR_E_ARG: return "invalid argument";
    case RADAR_E_UNSUPPORTED: return "unsupported size";
    case RADAR_E_WORKSPACE: return "workspace too small";
    case RADAR_E_HIP: return "HIP runtime error";
    case RADAR_E_NOT_COPRIME: return "ZC root not relatively prime to N";
    default: return "unknown status code";
  }
}

int radar_init(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RADAR_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return RADAR_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_init_mu);
  if (g_init_done[dev]) return RADAR_OK;
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      g_num_cus = cus;
  }
  // Every entry is exp(-2 pi i x/L) for some x < L, L a power of two <= LMAX;
  // it is taken from the same angle on the finest grid (LMAX points) in the
  // first quadrant, so equal angles get bit-identical entries.
  std::vector<double> qc(RADAR_TW_LMAX / 4 + 1), qs(RADAR_TW_LMAX / 4 + 1);
  for (int i = 0; i <= RADAR_TW_LMAX / 4; ++i) {
    const double ang = 2.0 * M_PI * (double)i / (double)RADAR_TW_LMAX;
    qc[i] = std::cos(ang);
    qs[i] = std::sin(ang);
  }
  auto w = [&](long long x, long long L) {  // W_L^x, any integer x
    const long long t = ((x % L + L) % L) * (RADAR_TW_LMAX / L);
    const int q = (int)(t / (RADAR_TW_LMAX / 4));
    const int rem = (int)(t % (RADAR_TW_LMAX / 4));
    const double c = qc[rem], sn = qs[rem];
    double re, im;  // exp(-i(2 pi rem/LMAX + q pi/2))
    switch (q) {
      case 0: re = c; im = -sn; break;
      case 1: re = -sn; im = -c; break;
      case 2: re = -c; im = sn; break;
      default: re = sn; im = c; break;
    }
    return make_float2((float)re, (float)im);
  };
  std::vector<float2> tab(RADAR_TW_ENTRIES, make_float2(0.0f, 0.0f));
  for (int L = 1; L <= RADAR_TW_LMAX; L <<= 1)
    for (int x = 0; x < L; ++x) tab[L + x] = w(x, L);
  for (int a = 0; a <= RADAR_TW_LOG2; ++a)
    for (int r = 1; r <= 4; ++r) {
      if (radar::stage_block(a, r) == 0) continue;
      const int NS = 1 << a, R = 1 << r, off = radar::stage_offset(a, r);
      for (int m = 0; m < R; ++m)
        for (int k = 0; k < NS; ++k) tab[off + m * NS + k] = w((long long)k * m, (long long)NS * R);
    }
  for (int n = 4; n <= 12; ++n)
    for (int p = 1; p <= 3; ++p) {
      const int N = 1 << n, F = 1 << p, off = radar::phase_offset(n, p);
      for (int b = 0; b < F; ++b)
        for (int k = 0; k < N; ++k) tab[off + b * N + k] = w((long long)k * b, (long long)F * N);
    }
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_radar_tw), tab.data(), tab.size() * sizeof(float2), 0,
                        hipMemcpyHostToDevice) != hipSuccess)
    return RADAR_E_HIP;
  // FP64 roots exp(+2 pi i x / 2^25), x = hi * 2^12 + lo, for the dense precoding stage
  std::vector<double2> r_hi(1 << (RADAR_ROOT64_LOG2 - 12)), r_lo(1 << 12);
  for (size_t i = 0; i < r_hi.size(); ++i) {
    const double ang = 2.0 * M_PI * (double)i / (double)r_hi.size();
    r_hi[i] = make_double2(std::cos(ang), std::sin(ang));
  }
  for (size_t i = 0; i < r_lo.size(); ++i) {
    const double ang = 2.0 * M_PI * (double)i / (double)(1 << RADAR_ROOT64_LOG2);
    r_lo[i] = make_double2(std::cos(ang), std::sin(ang));
  }
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_root64_hi), r_hi.data(), r_hi.size() * sizeof(double2), 0,
                        hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(g_root64_lo), r_lo.data(), r_lo.size() * sizeof(double2), 0,
                        hipMemcpyHostToDevice) != hipSuccess)
    return RADAR_E_HIP;
  // this device's copy of the allocation-free entry point's workspace
  void* sp = nullptr;
  if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || sp == nullptr) return RADAR_E_HIP;
  g_scratch_dev[dev] = sp;
  // the peak threshold kernel holds two words per row of the largest M' in LDS
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(radar::k_peak_threshold),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 2 * 16384 * (int)sizeof(uint32_t)) !=
      hipSuccess)
    return RADAR_E_HIP;
  g_init_done[dev] = true;
  return RADAR_OK;
}

int radar_simulate_frames(const radar_sim_desc* d, int32_t n_frames, const radar_cf32* A, int64_t frame_stride,
                          const radar_sim_target* targets, const int32_t* n_targets, const radar_cf32* noise,
                          radar_cf32* Y, uint32_t* status, void* hip_stream) {
  if (!d || !A || !targets || !n_targets || !Y) return RADAR_E_ARG;
  const int N = d->n_sub, M = d->n_sym;
  if (N <= 0 || M <= 0 || d->ld < N || d->n_guard < 0 || d->n_guard > N) return RADAR_E_ARG;
  if (d->max_targets < 1 || d->max_targets > 1024) return RADAR_E_ARG;
  if (!(d->fc_over_df > 0.0) || !std::isfinite(d->fc_over_df)) return RADAR_E_ARG;
  if (n_frames < 1 || n_frames > 65535) return RADAR_E_ARG;
  if (!is_pow2(N) || !is_pow2(M) || N < 16 || N > 4096 || M < 16 || M > 4096) return RADAR_E_UNSUPPORTED;
  const int64_t frame_elems = (int64_t)(M - 1) * d->ld + N;
  if (n_frames > 1 && frame_stride < frame_elems) return RADAR_E_ARG;
  int rc = ensure_init();
  if (rc != RADAR_OK) return rc;
  radar::SimArgs a{};
  a.A = reinterpret_cast<const float2*>(A);
  a.ld = d->ld;
  a.frame_stride = frame_stride;
  a.targets = targets;
  a.n_targets = n_targets;
  a.max_targets = d->max_targets;
  a.noise = reinterpret_cast<const float2*>(noise);
  a.Y = reinterpret_cast<float2*>(Y);
  a.status = status;
  a.M = M;
  a.n_guard = d->n_guard;
  a.fc_over_df = d->fc_over_df;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
#define SIM_CALL(n)                                                                              \
  {                                                                                              \
    constexpr int TEAMS = radar::kBlock / ((n) / 16);                                            \
    hipLaunchKernelGGL(radar::k_simulate<n>, dim3((M + TEAMS - 1) / TEAMS, n_frames), dim3(radar::kBlock), 0, s, a); \
  }
  RADAR_SIZE_SWITCH(N, SIM_CALL)
#undef SIM_CALL
  RADAR_HIP_CHECK(hipGetLastError());
  return RADAR_OK;
}

int radar_papr(int32_t n_sub, int32_t n_sym, int64_t ld, int32_t n_frames, const radar_cf32* A,
               int64_t frame_stride, float* papr, void* hip_stream) {
  const int N = n_sub, M = n_sym;
  if (!A || !papr || N <= 0 || M <= 0 || ld < N || n_frames < 1 || n_frames > 65535) return RADAR_E_ARG;
  if (!is_pow2(N) || !is_pow2(M) || N < 16 || N > 4096 || M < 16 || M > 4096) return RADAR_E_UNSUPPORTED;
  if (n_frames > 1 && frame_stride < (int64_t)(M - 1) * ld + N) return RADAR_E_ARG;
  int rc = ensure_init();
  if (rc != RADAR_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const float2* a = reinterpret_cast<const float2*>(A);
#define PAPR_CALL(n)                                                                                           \
  {                                                                                                            \
    constexpr int TEAMS = radar::kBlock / ((n) / 16);                                                          \
    hipLaunchKernelGGL(radar::k_papr<n>, dim3((M + TEAMS - 1) / TEAMS, n_frames), dim3(radar::kBlock), 0, s, a, \
                       ld, frame_stride, M, papr);                                                             \
  }
  RADAR_SIZE_SWITCH(N, PAPR_CALL)
#undef PAPR_CALL
  RADAR_HIP_CHECK(hipGetLastError());
  return RADAR_OK;
}

int radar_hpa(int32_t n_sub, int32_t n_sym, int64_t ld, int32_t n_frames, const radar_cf32* A, int64_t frame_stride,
              double q_db, radar_cf32* out, void* hip_stream) {
  const int N = n_sub, M = n_sym;
  if (!A || !out || N <= 0 || M <= 0 || ld < N || n_frames < 1 || n_frames > 65535 || !std::isfinite(q_db))
    return RADAR_E_ARG;
  if (!is_pow2(N) || !is_pow2(M) || N < 16 || N > 4096 || M < 16 || M > 4096) return RADAR_E_UNSUPPORTED;
  if (n_frames > 1 && frame_stride < (int64_t)(M - 1) * ld + N) return RADAR_E_ARG;
  int rc = ensure_init();
  if (rc != RADAR_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const float2* a = reinterpret_cast<const float2*>(A);
  float2* o = reinterpret_cast<float2*>(out);
  const float sat_factor = (float)std::pow(10.0, q_db / 10.0);
#define HPA_CALL(n)                                                                                           \
  {                                                                                                           \
    constexpr int TEAMS = radar::kBlock / ((n) / 16);                                                         \
    hipLaunchKernelGGL(radar::k_hpa<n>, dim3((M + TEAMS - 1) / TEAMS, n_frames), dim3(radar::kBlock), 0, s, a, \
                       o, ld, frame_stride, M, sat_factor);                                                   \
  }
  RADAR_SIZE_SWITCH(N, HPA_CALL)
#undef HPA_CALL
  RADAR_HIP_CHECK(hipGetLastError());
  return RADAR_OK;
}

int radar_tap_wiener_weights(const double* tap_power, int32_t n, double noise_var_tap, float* weights) {
  if (!tap_power || !weights || n < 1 || !(noise_var_tap >= 0.0) || !std::isfinite(noise_var_tap))
    return RADAR_E_ARG;
  for (int32_t i = 0; i < n; ++i)
    if (!(tap_power[i] >= 0.0) || !std::isfinite(tap_power[i])) return RADAR_E_ARG;
  for (int32_t i = 0; i < n; ++i) {
    const double p = tap_power[i], den = p + noise_var_tap;
    weights[i] = den > 0.0 ? (float)(p / den) : 0.0f;
  }
  return RADAR_OK;
}

size_t radar_frame_workspace_size(const radar_frame_desc* d, int32_t n_frames, int32_t k) {
  if (validate_desc(d) != RADAR_OK || n_frames < 1 || k < 1) return 0;
  return frame_ws_layout(d, n_frames, k).total;
}

static int check_frame_common(const radar_frame_desc* d, int32_t n_frames, int64_t frame_stride,
                              int64_t p_frame_stride, const void* P, bool p_optional = false) {
  const int rc = validate_desc(d);
  if (rc != RADAR_OK) return rc;
  if (n_frames < 1 || n_frames > 65535) return RADAR_E_ARG;
  const int64_t frame_elems = (int64_t)(d->n_sym - 1) * d->ld + d->n_sub;
  if (n_frames > 1 && frame_stride < frame_elems) return RADAR_E_ARG;
  if (!P) {
    if (!p_optional) return RADAR_E_ARG;
    return peaks_only_supported(d) ? RADAR_OK : RADAR_E_UNSUPPORTED;
  }
  if (reinterpret_cast<uintptr_t>(P) & 15) return RADAR_E_ARG;
  if (p_frame_stride % 4 != 0) return RADAR_E_ARG;
  if (n_frames > 1 && p_frame_stride < (int64_t)d->m_pad * d->n_pad) return RADAR_E_ARG;
  return RADAR_OK;
}

int radar_frame_process(const radar_frame_desc* d, int32_t n_frames, const radar_cf32* Y, const radar_cf32* A,
                        int64_t frame_stride, float* P, int64_t p_frame_stride, int32_t k, radar_peak* peaks,
                        int32_t* n_peaks, uint32_t* status, void* ws, size_t ws_bytes, void* hip_stream) {
  int rc = check_frame_common(d, n_frames, frame_stride, p_frame_stride, P, true);
  if (rc != RADAR_OK) return rc;
  if (!Y || !A || !peaks || !n_peaks || !status || !ws) return RADAR_E_ARG;
  if (k < 1 || k > 64) return RADAR_E_ARG;
  const FrameWs w = frame_ws_layout(d, n_frames, k);
  if (ws_bytes < w.total) return RADAR_E_WORKSPACE;
  if ((rc = ensure_init()) != RADAR_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(radar::k0_clear, dim3((n_frames + 255) / 256), dim3(256), 0, s, status, n_peaks, n_frames,
                     nullptr);
  RADAR_HIP_CHECK(hipGetLastError());
  char* wsb = static_cast<char*>(ws);
  rc = enqueue_transforms(d, n_frames, reinterpret_cast<const float2*>(Y), reinterpret_cast<const float2*>(A),
                          frame_stride, 0, P, p_frame_stride, status, w, wsb, s);
  if (rc != RADAR_OK) return rc;
  const bool thr = (d->flags & RADAR_FLAG_THRESHOLD) != 0;
  rc = enqueue_peaks(P, p_frame_stride, d->m_pad, d->n_pad, n_frames, k, w.pk, wsb, peaks, n_peaks, s, nullptr,
                     thr ? reinterpret_cast<const float*>(wsb + w.inv_sum) : nullptr, d->n_sym,
                     thr ? eta_factor_of(d) : 0.0f, d, reinterpret_cast<const float2*>(wsb + w.U),
                     reinterpret_cast<float*>(wsb + w.ring));
  if (rc != RADAR_OK || !(d->flags & RADAR_FLAG_REFINE)) return rc;
  return enqueue_refine(d, n_frames, k, reinterpret_cast<const float2*>(wsb + w.taps), peaks, n_peaks, nullptr, s);
}

int radar_frame_process_noalloc(const radar_frame_desc* d, int32_t n_frames, const radar_cf32* Y,
                                const radar_cf32* A, int64_t frame_stride, float* P, int64_t p_frame_stride,
                                int32_t k, radar_peak* peaks, int32_t* n_peaks, uint32_t* status,
                                void* hip_stream) {
  int rc = check_frame_common(d, n_frames, frame_stride, p_frame_stride, P, true);
  if (rc != RADAR_OK) return rc;
  if (k < 1 || k > 64) return RADAR_E_ARG;
  const size_t need = frame_ws_layout(d, n_frames, k).total;
  if (need > (size_t)RADAR_NOALLOC_WS_BYTES) return RADAR_E_WORKSPACE;
  if ((rc = ensure_init()) != RADAR_OK) return rc;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RADAR_E_HIP;
  // ensure_init has run on this device, so its scratch address is known; the
  // path clears what it needs itself (status and peak counts by a fill
  // kernel, every workspace word is written before it is read)
  return radar_frame_process(d, n_frames, Y, A, frame_stride, P, p_frame_stride, k, peaks, n_peaks, status,
                             g_scratch_dev[dev], need, hip_stream);
}

int radar_periodogram(const radar_frame_desc* d, int32_t n_frames, const radar_cf32* H, int64_t frame_stride,
                      float* P, int64_t p_frame_stride, void* ws, size_t ws_bytes, void* hip_stream) {
  int rc = check_frame_common(d, n_frames, frame_stride, p_frame_stride, P);
  if (rc != RADAR_OK) return rc;
  if (!H || !ws || (d->flags & (RADAR_FLAG_REFINE | RADAR_FLAG_THRESHOLD))) return RADAR_E_ARG;
  if (d->zc_mode != RADAR_ZC_NONE) return RADAR_E_ARG;
  const FrameWs w = frame_ws_layout(d, n_frames, 1);
  if (ws_bytes < w.total) return RADAR_E_WORKSPACE;
  if ((rc = ensure_init()) != RADAR_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  return enqueue_transforms(d, n_frames, reinterpret_cast<const float2*>(H), nullptr, frame_stride, 1, P,
                            p_frame_stride, nullptr, w, static_cast<char*>(ws), s);
}

size_t radar_detect_workspace_size(int32_t m_pad, int32_t n_pad, int32_t n_frames, int32_t k) {
  if (m_pad < 4 || n_pad < 4 || !is_pow2(m_pad) || !is_pow2(n_pad) || m_pad > 16384 || n_pad > 16384 ||
      n_frames < 1 || k < 1)
    return 0;
  return peak_ws_layout(m_pad, n_frames, k, 0).total;
}

int radar_detect_topk(const float* P, int32_t m_pad, int32_t n_pad, int32_t n_frames, int64_t p_frame_stride,
                      int32_t k, radar_peak* peaks, int32_t* n_peaks, void* ws, size_t ws_bytes,
                      void* hip_stream) {
  if (!P || !peaks || !n_peaks || !ws) return RADAR_E_ARG;
  if (m_pad < 4 || n_pad < 4 || !is_pow2(m_pad) || !is_pow2(n_pad)) return RADAR_E_UNSUPPORTED;
  if (m_pad > 16384 || n_pad > 16384) return RADAR_E_UNSUPPORTED;
  if (n_frames < 1 || n_frames > 65535 || k < 1 || k > 64) return RADAR_E_ARG;
  if (n_frames > 1 && p_frame_stride < (int64_t)m_pad * n_pad) return RADAR_E_ARG;
  if (ws_bytes < radar_detect_workspace_size(m_pad, n_pad, n_frames, k)) return RADAR_E_WORKSPACE;
  const int rc = ensure_init();
  if (rc != RADAR_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(radar::k0_clear, dim3((n_frames + 255) / 256), dim3(256), 0, s, nullptr, n_peaks, n_frames,
                     nullptr);
  RADAR_HIP_CHECK(hipGetLastError());
  const PeakWs w = peak_ws_layout(m_pad, n_frames, k, 0);
  char* wsb = static_cast<char*>(ws);
  hipLaunchKernelGGL(radar::k_row_max, dim3(m_pad, n_frames), dim3(256), 0, s, P, p_frame_stride, m_pad, n_pad,
                     reinterpret_cast<float*>(wsb + w.rowmax), nullptr);
  RADAR_HIP_CHECK(hipGetLastError());
  return enqueue_peaks(P, p_frame_stride, m_pad, n_pad, n_frames, k, w, wsb, peaks, n_peaks, s);
}

void radar_sft_default(radar_sft_desc* s, int32_t k) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  static const int dirs[8][2] = {{1, 1}, {1, -1}, {1, 2}, {2, 1}, {1, -2}, {2, -1}, {1, 0}, {0, 1}};
  s->n_dirs = 8;
  for (int i = 0; i < 8; ++i) {
    s->dirs[i][0] = dirs[i][0];
    s->dirs[i][1] = dirs[i][1];
  }
  s->k = k;
  s->pfa = 1e-2f;
  s->tol = 0.25f;
}

size_t radar_fps_sft_workspace_size(const radar_frame_desc* d, const radar_sft_desc* sd, int32_t n_frames) {
  SftPlan p;
  if (validate_sft(d, sd, &p) != RADAR_OK || n_frames < 1) return 0;
  return p.general ? sft_general_ws(p, n_frames).total : sft_spectra_bytes(p, n_frames);
}

int radar_fps_sft(const radar_frame_desc* d, const radar_sft_desc* sd, int32_t n_frames, const radar_cf32* Y,
                  const radar_cf32* A, int64_t frame_stride, radar_peak* peaks, int32_t* n_peaks,
                  uint32_t* status, radar_cf32* slices, void* ws, size_t ws_bytes, void* hip_stream) {
  SftPlan p;
  int rc = validate_sft(d, sd, &p);
  if (rc != RADAR_OK) return rc;
  if (n_frames < 1 || n_frames > 65535) return RADAR_E_ARG;
  if (!Y || !A || !peaks || !n_peaks || !status) return RADAR_E_ARG;
  const int64_t frame_elems = (int64_t)(p.M - 1) * d->ld + p.N;
  if (n_frames > 1 && frame_stride < frame_elems) return RADAR_E_ARG;
  float2* spectra = reinterpret_cast<float2*>(slices);
  if (p.general) {
    // pass 1's output and the tables need the workspace even when the caller takes the spectra
    if (!ws) return RADAR_E_ARG;
    if (ws_bytes < sft_general_ws(p, n_frames).total) return RADAR_E_WORKSPACE;
    if (!spectra) spectra = static_cast<float2*>(ws);
  } else if (!spectra) {
    if (!ws) return RADAR_E_ARG;
    if (ws_bytes < sft_spectra_bytes(p, n_frames)) return RADAR_E_WORKSPACE;
    spectra = static_cast<float2*>(ws);
  }
  if ((rc = ensure_init()) != RADAR_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(radar::k0_clear, dim3((n_frames + 255) / 256), dim3(256), 0, s, status, n_peaks, n_frames,
                     nullptr);
  RADAR_HIP_CHECK(hipGetLastError());

  radar::K5Args a5{};
  a5.Y = reinterpret_cast<const float2*>(Y);
  a5.A = reinterpret_cast<const float2*>(A);
  a5.ld = d->ld;
  a5.frame_stride = frame_stride;
  a5.S = spectra;
  a5.status = status;
  a5.N = p.N;
  a5.M = p.M;
  a5.n_dirs = p.n_dirs;
  a5.total = n_frames * p.n_dirs * 3;
  a5.zc_root = d->zc_mode == RADAR_ZC_DIAG ? (uint32_t)d->zc_root : 0u;
  a5.zc_shift = d->zc_mode == RADAR_ZC_DIAG ? (uint32_t)d->zc_shift : 0u;
  radar::K6Args a6{};
  a6.S = spectra;
  a6.peaks = peaks;
  a6.n_peaks = n_peaks;
  a6.N = p.N;
  a6.M = p.M;
  a6.n_dirs = p.n_dirs;
  a6.k = sd->k;
  a6.thr_factor = (float)(-std::log((double)sd->pfa) / std::log(2.0));
  a6.tol = sd->tol;
  a6.floor_rel = 1e-10f;
  for (int i = 0; i < p.n_dirs; ++i) {
    a5.dir_a[i] = a6.dir_a[i] = p.dir_a[i];
    a5.dir_b[i] = a6.dir_b[i] = p.dir_b[i];
  }
  if (p.general) {
    char* wsb = static_cast<char*>(ws);
    const SftGeneralWs w = sft_general_ws(p, n_frames);
    radar::K5gArgs g{};
    g.Y = a5.Y;
    g.A = a5.A;
    g.ld = a5.ld;
    g.frame_stride = a5.frame_stride;
    const bool zc_on = d->zc_mode == RADAR_ZC_DIAG;
    g.zc = zc_on ? reinterpret_cast<float2*>(wsb + w.zc) : nullptr;
    g.wr = reinterpret_cast<float2*>(wsb + w.wr);
    g.Z = reinterpret_cast<float2*>(wsb + w.Z);
    g.S = spectra;
    g.status = status;
    g.N = p.N;
    g.M = p.M;
    g.Q = p.Q;
    g.P = p.P;
    g.R = p.R;
    g.n_dirs = p.n_dirs;
    g.total = a5.total;
    g.r_inv = p.r_inv;
    g.p_inv = p.p_inv;
    radar::K6gArgs g6{};
    g6.S = spectra;
    g6.peaks = peaks;
    g6.n_peaks = n_peaks;
    g6.N = p.N;
    g6.M = p.M;
    g6.Q = p.Q;
    g6.n_dirs = p.n_dirs;
    g6.k = sd->k;
    g6.nm_over_q = (float)p.gcd_nm;
    g6.thr_factor = a6.thr_factor;
    g6.tol = a6.tol;
    g6.floor_rel = a6.floor_rel;
    for (int i = 0; i < p.n_dirs; ++i) {
      g.dir_a[i] = g6.dir_a[i] = p.dir_a[i];
      g.dir_b[i] = g6.dir_b[i] = p.dir_b[i];
    }
    const int64_t two_n = 2 * (int64_t)p.N;
    const int64_t root = zc_on ? ((d->zc_root % two_n) + two_n) % two_n : 0;
    const int64_t shift = zc_on ? ((d->zc_shift % two_n) + two_n) % two_n : 0;
    return launch_sft_general(g, g6, root, shift, n_frames, s);
  }
  switch (p.Q) {
    case 16: return launch_sft_q<16>(a5, a6, n_frames, s);
    case 32: return launch_sft_q<32>(a5, a6, n_frames, s);
    case 64: return launch_sft_q<64>(a5, a6, n_frames, s);
    case 128: return launch_sft_q<128>(a5, a6, n_frames, s);
    case 256: return launch_sft_q<256>(a5, a6, n_frames, s);
    case 512: return launch_sft_q<512>(a5, a6, n_frames, s);
    case 1024: return launch_sft_q<1024>(a5, a6, n_frames, s);
    case 2048: return launch_sft_q<2048>(a5, a6, n_frames, s);
    case 4096: return launch_sft_q<4096>(a5, a6, n_frames, s);
    default: return RADAR_E_UNSUPPORTED;
  }
}

size_t radar_batch_workspace_size(const radar_frame_job* jobs, int32_t n_jobs) {
  if (!jobs || n_jobs < 1) return 0;
  for (int i = 0; i < n_jobs; ++i)
    if (validate_desc(&jobs[i].d) != RADAR_OK || jobs[i].k < 1 || jobs[i].k > 64) return 0;
  std::vector<BatchGroup> groups;
  return plan_groups(jobs, n_jobs, groups);
}

int radar_batch_create(const radar_frame_job* jobs, int32_t n_jobs, int32_t flags, void* ws, size_t ws_bytes,
                       void* hip_stream, radar_batch** out) {
  if (!out || !jobs || n_jobs < 1 || !ws) return RADAR_E_ARG;
  *out = nullptr;
  if (flags & ~(RADAR_BATCH_GRAPH | RADAR_BATCH_TUNE)) return RADAR_E_ARG;
  for (int i = 0; i < n_jobs; ++i) {
    const int rc = validate_job(jobs[i]);
    if (rc != RADAR_OK) return rc;
  }
  auto* b = new radar_batch();
  const size_t need = plan_groups(jobs, n_jobs, b->groups);
  if (ws_bytes < need) {
    delete b;
    return RADAR_E_WORKSPACE;
  }
  b->ws = static_cast<char*>(ws);
  b->flags = flags;
  int rc = ensure_init();
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  // job tables, uploaded once
  for (const auto& g : b->groups) {
    if (rc != RADAR_OK) break;
    std::vector<radar::FrameRef> refs(g.jobs.size());
    for (size_t j = 0; j < g.jobs.size(); ++j) {
      const radar_frame_job& jb = jobs[g.jobs[j]];
      refs[j] = {reinterpret_cast<const float2*>(jb.Y), reinterpret_cast<const float2*>(jb.A), jb.P, jb.peaks,
                 jb.n_peaks, jb.status, (jb.d.flags & RADAR_FLAG_THRESHOLD) ? eta_factor_of(&jb.d) : 0.0f};
    }
    if (hipMemcpyAsync(b->ws + g.refs_off, refs.data(), refs.size() * sizeof(radar::FrameRef),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = RADAR_E_HIP;
  }
  if (rc == RADAR_OK && (flags & RADAR_BATCH_TUNE))
    for (auto& g : b->groups)
      if ((rc = tune_group(*b, g, s)) != RADAR_OK) break;
  if (rc == RADAR_OK && (flags & RADAR_BATCH_GRAPH)) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
      rc = RADAR_E_HIP;
    } else {
      // groups run on up to kBatchBranches concurrent branches (each has its
      // own workspace region), heaviest first onto the least loaded branch
      const int nb = std::min<int>(kBatchBranches, (int)b->groups.size());
      std::vector<hipStream_t> br(nb, nullptr);
      std::vector<hipEvent_t> ev(nb + 1, nullptr);
      for (int i = 0; i < nb && rc == RADAR_OK; ++i)
        if (hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking) != hipSuccess) rc = RADAR_E_HIP;
      for (int i = 0; i <= nb && rc == RADAR_OK; ++i)
        if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) rc = RADAR_E_HIP;
      std::vector<int> order(b->groups.size());
      for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
      // the measured time of each group when the batch was tuned, else its
      // algorithmic bytes
      bool timed = true;
      for (const auto& g : b->groups) timed = timed && g.tune.ms > 0.0f;
      const auto cost = [&](int x) { return timed ? (double)b->groups[x].tune.ms : b->groups[x].work; };
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
      g_capturing = true;
      if (rc == RADAR_OK && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
        rc = RADAR_E_HIP;
      if (rc == RADAR_OK && hipEventRecord(ev[nb], cs) != hipSuccess) rc = RADAR_E_HIP;
      for (int i = 0; i < nb && rc == RADAR_OK; ++i)
        if (hipStreamWaitEvent(br[i], ev[nb], 0) != hipSuccess) rc = RADAR_E_HIP;
      std::vector<double> load(nb, 0.0);
      for (int gi : order) {
        if (rc != RADAR_OK) break;
        const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[j] += cost(gi);
        rc = enqueue_group(*b, b->groups[gi], br[j]);
      }
      for (int i = 0; i < nb && rc == RADAR_OK; ++i) {
        if (hipEventRecord(ev[i], br[i]) != hipSuccess || hipStreamWaitEvent(cs, ev[i], 0) != hipSuccess)
          rc = RADAR_E_HIP;
      }
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(cs, &graph);
      g_capturing = false;
      if (rc == RADAR_OK && ec != hipSuccess) rc = RADAR_E_HIP;
      b->graph = graph;
      if (rc == RADAR_OK && hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0) != hipSuccess)
        rc = RADAR_E_HIP;
      for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
      for (auto st : br)
        if (st) (void)hipStreamDestroy(st);
      (void)hipStreamDestroy(cs);
    }
  }
  if (rc != RADAR_OK) {
    radar_batch_destroy(b);
    return rc;
  }
  *out = b;
  return RADAR_OK;
}

int radar_batch_launch(radar_batch* b, void* hip_stream) {
  if (!b) return RADAR_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if (b->exec) return hipGraphLaunch(b->exec, s) == hipSuccess ? RADAR_OK : RADAR_E_HIP;
  for (const auto& g : b->groups) {
    const int rc = enqueue_group(*b, g, s);
    if (rc != RADAR_OK) return rc;
  }
  return RADAR_OK;
}

int radar_batch_info(const radar_batch* b, int32_t g, int32_t* n_groups, int32_t* n_frames, int32_t* k1_mult,
                     int32_t* k3_mult, int32_t* k3_generic) {
  if (!b) return RADAR_E_ARG;
  if (n_groups) *n_groups = (int32_t)b->groups.size();
  if (g < 0 || g >= (int32_t)b->groups.size()) return (n_frames || k1_mult || k3_mult || k3_generic) ? RADAR_E_ARG : RADAR_OK;
  const BatchGroup& gr = b->groups[g];
  if (n_frames) *n_frames = (int32_t)gr.jobs.size();
  if (k1_mult) *k1_mult = gr.tune.k1_mult;
  if (k3_mult) *k3_mult = gr.tune.k3_mult;
  if (k3_generic) *k3_generic = gr.tune.k3_generic ? 1 : 0;
  return RADAR_OK;
}

int radar_batch_plan(const radar_batch* b, int32_t g, int32_t* k2_half_tile, int32_t* scan_groups) {
  if (!b || g < 0 || g >= (int32_t)b->groups.size()) return RADAR_E_ARG;
  const Tuning& t = b->groups[g].tune;
  if (k2_half_tile) *k2_half_tile = t.k2_half ? 1 : 0;
  if (scan_groups) *scan_groups = t.scan_groups;
  return RADAR_OK;
}

void radar_batch_destroy(radar_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
}

int32_t radar_cnn_param_count(void) { return radar::kCnnParams; }

size_t radar_cnn_workspace_size(int32_t batch, int32_t train) {
  if (batch < 1 || batch > 65536) return 0;
  return cnn_ws_layout(batch, train != 0).total;
}

int radar_cnn_patches(const float* P, int64_t p_frame_stride, int32_t m_pad, int32_t n_pad, int32_t n_frames,
                      int32_t k, const radar_peak* peaks, const int32_t* n_peaks, float* patches, int32_t* valid,
                      void* hip_stream) {
  if (!P || !peaks || !n_peaks || !patches) return RADAR_E_ARG;
  if (n_frames < 1 || k < 1 || k > 64 || (int64_t)n_frames * k > 65535 * 16) return RADAR_E_ARG;
  if (!is_pow2(m_pad) || !is_pow2(n_pad) || m_pad < 32 || n_pad < 32 || m_pad > 16384 || n_pad > 16384)
    return RADAR_E_UNSUPPORTED;
  if (n_frames > 1 && p_frame_stride < (int64_t)m_pad * n_pad) return RADAR_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(radar::k_cnn_patches, dim3(n_frames * k), dim3(256), 0, s, P, p_frame_stride, m_pad, n_pad, k,
                     peaks, n_peaks, patches, valid);
  RADAR_HIP_CHECK(hipGetLastError());
  return RADAR_OK;
}

int radar_cnn_forward(const float* theta, const float* patches, int32_t batch, float* out, void* ws, size_t ws_bytes,
                      void* hip_stream) {
  if (!theta || !patches || !out || !ws || batch < 1 || batch > 65536) return RADAR_E_ARG;
  const CnnWs w = cnn_ws_layout(batch, false);
  if (ws_bytes < w.total) return RADAR_E_WORKSPACE;
  int rc = ensure_init();  // the CU count sizes the persistent grid
  if (rc == RADAR_OK) rc = cnn_setup();
  if (rc != RADAR_OK) return rc;
  return cnn_forward_fused(theta, patches, batch, w, static_cast<char*>(ws), out,
                           reinterpret_cast<hipStream_t>(hip_stream));
}

int radar_cnn_gradient(const float* theta, const float* patches, const float* labels, int32_t batch, float* grad,
                       float* loss, void* ws, size_t ws_bytes, void* hip_stream) {
  if (!theta || !patches || !labels || !grad || !ws || batch < 1 || batch > 65536) return RADAR_E_ARG;
  const CnnWs w = cnn_ws_layout(batch, true);
  if (ws_bytes < w.total) return RADAR_E_WORKSPACE;
  int rc = cnn_setup();
  if (rc != RADAR_OK) return rc;
  return cnn_gradient(theta, patches, labels, batch, w, static_cast<char*>(ws), grad, loss,
                      reinterpret_cast<hipStream_t>(hip_stream));
}

int radar_cnn_adam(float* theta, const float* grad, float* m, float* v, int32_t step, float lr, void* hip_stream) {
  if (!theta || !grad || !m || !v || step < 1 || !(lr > 0.0f)) return RADAR_E_ARG;
  return cnn_adam(theta, grad, m, v, step, lr, reinterpret_cast<hipStream_t>(hip_stream));
}

int radar_cnn_train_step(float* theta, float* m, float* v, int32_t step, float lr, const float* patches,
                         const float* labels, int32_t batch, float* loss, void* ws, size_t ws_bytes,
                         void* hip_stream) {
  if (!theta || !m || !v || !patches || !labels || !ws || batch < 1 || batch > 65536 || step < 1 || !(lr > 0.0f))
    return RADAR_E_ARG;
  const CnnWs w = cnn_ws_layout(batch, true);
  if (ws_bytes < w.total) return RADAR_E_WORKSPACE;
  int rc = cnn_setup();
  if (rc != RADAR_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  char* wsb = static_cast<char*>(ws);
  float* grad = reinterpret_cast<float*>(wsb + w.grad);
  rc = cnn_gradient(theta, patches, labels, batch, w, wsb, grad, loss, s);
  if (rc != RADAR_OK) return rc;
  return cnn_adam(theta, grad, m, v, step, lr, s);
}

int radar_timing_start(int32_t max_launches) {
  if (max_launches < 1 || max_launches > (1 << 20)) return RADAR_E_ARG;
  if (g_timer.on) return RADAR_E_ARG;
  for (int st = 0; st < RADAR_NUM_STAGES; ++st) {
    g_timer.ev[st].assign(2 * (size_t)max_launches, nullptr);
    for (auto& e : g_timer.ev[st])
      if (hipEventCreate(&e) != hipSuccess) return RADAR_E_HIP;
    g_timer.used[st] = 0;
  }
  g_timer.cap = max_launches;
  g_timer.on = true;
  return RADAR_OK;
}

int radar_timing_stop(double* ms_total, int64_t* launches) {
  if (!g_timer.on) return RADAR_E_ARG;
  g_timer.on = false;
  int rc = RADAR_OK;
  for (int st = 0; st < RADAR_NUM_STAGES; ++st) {
    double tot = 0.0;
    for (int i = 0; i < g_timer.used[st]; ++i) {
      float ms = 0.0f;
      if (hipEventSynchronize(g_timer.ev[st][2 * i + 1]) != hipSuccess ||
          hipEventElapsedTime(&ms, g_timer.ev[st][2 * i], g_timer.ev[st][2 * i + 1]) != hipSuccess)
        rc = RADAR_E_HIP;
      tot += ms;
    }
    if (ms_total) ms_total[st] = tot;
    if (launches) launches[st] = g_timer.used[st];
    for (auto& e : g_timer.ev[st])
      if (e) (void)hipEventDestroy(e);
    g_timer.ev[st].clear();
    g_timer.used[st] = 0;
  }
  return rc;
}

}  // extern "C"
