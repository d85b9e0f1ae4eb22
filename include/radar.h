/*
 * radar.h -- C ABI of the MI355X (gfx950) OFDM monostatic radar receive path.
 *
 * The operations follow Delamou, Noubir, Dang, Amhoud, "An Efficient
 * OFDM-Based Monostatic Radar Design for Multitarget Detection" (arXiv
 * 2209.03883):
 *   - Zadoff-Chu de-precoding (Sec. III-B, Eq. 23-24),
 *   - spectral division / LS channel estimate (Sec. II-B.2, Eq. 16),
 *   - DFT-CE denoising (Sec. III-A, Eq. 20-22),
 *   - the windowed, zero-padded 2D periodogram (Sec. II-B.2, Eq. 17),
 *   - extraction of its dominant peaks (Sec. II-B.2, Eq. 17-19).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.   Every array pointer is a DEVICE pointer owned by the caller
 *           (for example a torch CUDA tensor).  Descriptors and the
 *           radar_frame_desc struct are HOST pointers, read before the call
 *           returns.  The library never allocates device memory inside a call:
 *           scratch space is the caller's workspace `ws` of `ws_bytes` bytes,
 *           sized by the matching *_workspace_size function.  The library's
 *           only own device state is a read-only twiddle table, written once
 *           per device by radar_init() (called implicitly by the first entry
 *           point that runs on that device).
 * Layout.   A frame is symbol-major: element (l, k) -- OFDM symbol l,
 *           subcarrier k -- sits at  base + l*ld + k  (ld >= N).  Frame f of a
 *           batch starts `frame_stride` elements after frame f-1.  The
 *           periodogram P of a frame is float32 [M'][N'] row-major; row
 *           s + M'/2 holds the signed Doppler index s in [-M'/2, M'/2) and
 *           column r in [0, N') the range index.
 * Streams.  `hip_stream` is a hipStream_t (NULL = the default stream).
 *           Calls validate on the host, enqueue kernels and return; the
 *           caller synchronises.  Calls on distinct streams with distinct
 *           workspaces may run concurrently.
 * Errors.   A negative return means the arguments were rejected and nothing
 *           was enqueued (RADAR_E_*).  Data-dependent problems found on the
 *           device (a zero transmitted symbol, a non-finite input) set bits in
 *           the frame's `status` word (RADAR_ST_*); that frame's outputs are
 *           then undefined, the others are unaffected.  Nothing throws across
 *           this boundary.
 * Sizes.    N, M: powers of two in [16, 4096].  N' = N * {1,2,4,8};
 *           M' = M * 2^j with M' <= 16384.  1 <= n_cp <= N.
 */
#ifndef RADAR_H
#define RADAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  float re, im;                 /* same layout as torch.complex64 / hipFloatComplex */
} radar_cf32;

enum {
  RADAR_OK = 0,
  RADAR_E_ARG = -1,             /* null pointer, bad size, bad stride, bad enum */
  RADAR_E_UNSUPPORTED = -2,     /* a size this build does not implement */
  RADAR_E_WORKSPACE = -3,       /* ws_bytes smaller than the *_workspace_size result */
  RADAR_E_HIP = -4,             /* a HIP runtime call failed */
  RADAR_E_NOT_COPRIME = -5      /* ZC root not relatively prime to N (Sec. III-B) */
};

enum { RADAR_WIN_RECT = 0, RADAR_WIN_HANN = 1, RADAR_WIN_HAMMING = 2 };  /* periodic windows */
/* ZC precoding (Sec. III-B).  DIAG: each subcarrier k carries z_k a_k, z the
 * length-N sequence of Eq. 23.  DENSE: Eq. 24 read literally with L = N^2,
 * each symbol carries a_p = Z_m a / sqrt(N), Z_m[i][j] = zc_L(i N + j). */
enum { RADAR_ZC_NONE = 0, RADAR_ZC_DIAG = 1, RADAR_ZC_DENSE = 2 };
enum { RADAR_ST_ZERO_SYMBOL = 1u, RADAR_ST_NONFINITE = 2u,
       RADAR_ST_ISI = 4u /* radar_simulate_frames: a target's delay left [0, n_guard] */ };
/* radar_frame_desc.flags */
enum {
  RADAR_FLAG_REFINE = 1,   /* sub-cell refinement of the peaks (radar_frame_process) */
  RADAR_FLAG_BF16X3 = 2,   /* Doppler and range FFTs' radix-16 stages on BF16 matrix cores, split operands */
  RADAR_FLAG_FP16X3 = 4,   /* the same with FP16 operands and power-of-two scaling */
  RADAR_FLAG_THRESHOLD = 8,/* keep only peaks at or above the detection threshold of Eq. 18 */
  RADAR_FLAG_FP16 = 16     /* range stage on FP16 matrix cores, operands rounded once (N = 1024 only) */
};

/* One frame shape.  Names follow the paper: N subcarriers, M OFDM symbols,
 * N' >= N and M' >= M the zero-padded periodogram sizes of Eq. 17, N_cp the
 * DFT-CE taps kept by Eq. 21 (n_cp == N disables DFT-CE, i.e. plain LS-CE). */
typedef struct {
  int32_t n_sub;                /* N  */
  int32_t n_sym;                /* M  */
  int32_t n_pad;                /* N' */
  int32_t m_pad;                /* M' */
  int32_t n_cp;                 /* N_cp */
  int32_t zc_mode;              /* RADAR_ZC_* */
  int32_t zc_root;              /* r' of Eq. 23, relatively prime to N (and so to N^2) */
  int32_t zc_shift;             /* q' of Eq. 23, any integer */
  int32_t window;               /* RADAR_WIN_*, applied separably over k and l */
  int32_t flags;                /* RADAR_FLAG_* bits, 0 for none */
  int64_t ld;                   /* elements between consecutive OFDM symbols, >= N */
  float pfa;                    /* RADAR_FLAG_THRESHOLD: false-alarm probability per cell, (0, 1) */
  float noise_power;            /* RADAR_FLAG_THRESHOLD: noise power sigma^2 per received element, > 0 */
  const float *tap_weights;     /* device, n_cp floats g(n) scaling the kept DFT-CE taps (LMMSE-based
                                   DFT-CE, Sec. III-A / Fig. 5; see radar_tap_wiener_weights), or NULL
                                   for plain DFT-CE; 4-byte aligned, caller-owned */
} radar_frame_desc;

/* One detected peak of P.  s is the signed Doppler index (row - M'/2), r the
 * range index, p = P[s + M'/2][r].  s_off / r_off are sub-cell refinements
 * (0 unless a refinement entry point filled them). */
typedef struct {
  int32_t s, r;
  float p;
  float s_off, r_off;
} radar_peak;

/* Library version (major*10000 + minor*100 + patch). */
int radar_version(void);

/* Human-readable text for a RADAR_* return code. */
const char *radar_status_string(int code);

/* Upload the twiddle table to the current HIP device.  Idempotent and
 * thread-safe; entry points call it themselves.  Call it once outside any
 * stream capture before capturing radar calls into a graph. */
int radar_init(void);

/* ------------------------------------------------------------------------
 * radar_frame_process -- the whole receive path for a batch of frames.
 *
 * For each frame f < n_frames (all sharing *d):
 *   H = Y / (z_k * A)                 Eq. 16 with ZC de-precoding (Sec. III-B,
 *                                     z = Eq. 23 sequence, diagonal reading)
 *   or H = Y / A_p, A_p = Z_m A / sqrt(N) per symbol (RADAR_ZC_DENSE): the
 *                                     receiver forms A_p from A as D1 F D2 (two
 *                                     diagonals around an N-point DFT), one
 *                                     extra FFT per symbol
 *   H' = DFT_N(trunc_{N_cp}(IDFT_N(H)))   per symbol (Eq. 20-22); with
 *                                     d->tap_weights, kept tap n is scaled by
 *                                     tap_weights[n] (LMMSE-based DFT-CE)
 *   P  = Eq. 17 on H' with the separable periodic window, zero padded to
 *        N' x M', scaled by 1/(N M)
 *   peaks = the k largest 3x3 cyclic local maxima of P, ranked by
 *           (P descending, flat index row*N'+r ascending).
 *   With RADAR_FLAG_REFINE each peak also gets sub-cell offsets (s_off,
 *   r_off, in cells of the N' x M' grid): the 16x-padded periodogram is
 *   evaluated on the 7 x 7 fine cells around the peak directly from the DFT-CE
 *   taps (FP32 Doppler sums, FP64 range sums), the best fine cell of the inner
 *   5 x 5 is taken and a least-squares quadratic of ln P through its 3 x 3
 *   neighbourhood is solved in FP64 (separable parabolas when that quadratic
 *   has no maximum within one cell); offsets are clamped to half a fine cell
 *   about the best fine cell.  Needs M'/M <= 16, N'/N <= 16 and M <= 1024.
 *   With RADAR_FLAG_BF16X3 or RADAR_FLAG_FP16X3 the FFT butterflies run as
 *   DFTs by matrix product on the matrix cores: data and DFT matrix are each
 *   split into two half-precision parts (v = hi + lo, hi = rn(v),
 *   lo = rn(v - hi)), the products hi*hi, hi*lo and lo*hi accumulate in FP32;
 *   twiddles, windows, the taps stage and |.|^2 stay FP32.  At N = 1024 with
 *   P written, the whole range stage (DFT back, window, padded range IDFT) is
 *   two passes of 32-point DFTs per transform, each row scaled by a power of
 *   two into the half-precision range, and the Doppler stage stays FP32; at
 *   other N (and with P = NULL) the radix-16 stages of the Doppler FFT and of
 *   the range IFFTs run as 16-point DFTs.  These forms exist for N' = 4N,
 *   4 N_cp <= N, N >= 256 (RADAR_E_UNSUPPORTED otherwise).
 *   With RADAR_FLAG_FP16 the range stage is the N = 1024 matrix-core form
 *   above with each operand rounded once to FP16 (one product per pass, a
 *   third of the matrix-core work): the periodogram's normwise error is of
 *   the order of 1e-4 instead of 1e-7.  Only for N = 1024, N' = 4N,
 *   4 N_cp <= N (RADAR_E_UNSUPPORTED otherwise).  With P = NULL the form's
 *   row maxima only choose the rows to scan, and those rows are recomputed
 *   in FP32: the peaks are the FP32 periodogram's.
 *   At most one of RADAR_FLAG_BF16X3, RADAR_FLAG_FP16X3, RADAR_FLAG_FP16.
 *   With RADAR_FLAG_THRESHOLD the peaks are the paper's detections (Eq. 18):
 *   local maxima with P >= eta = -ln(pfa) sigma_P^2, at most k, where
 *   sigma_P^2 = noise_power * mean(1/|a|^2) * sum_l w_l^2 * sum_k w_k^2 / (N M)
 *   is the mean noise power of a cell inside the cyclic-prefix range box (the
 *   LS estimate's noise through DFT-CE and the windowed transform; the mean
 *   of 1/|a|^2 over the frame is taken from A by the taps stage).  n_peaks
 *   counts only those detections.
 * Y, A:     input frames, frame f at Y + f*frame_stride (elements).
 * P:        output, frame f at P + f*p_frame_stride (floats);
 *           p_frame_stride >= M'*N' and a multiple of 4; P 16-byte aligned.
 *           NULL: peaks only, P is not materialised (p_frame_stride ignored).
 *           The range stage then keeps only its row maxima, and the peak
 *           search recomputes the rows it scans and their neighbours with
 *           the range stage's own row code, compiled into a second kernel:
 *           a recomputed cell may differ from the written one by a few FP32
 *           ulps (the compiler may order a multiply-add differently), so the
 *           peaks match those found with P written except at near-ties.  The
 *           rows are listed twice: first those whose maximum reaches the
 *           bound of the row maxima, then, from the k-th candidate found,
 *           any other row that can still hold a top-k peak given the error
 *           of the maxima (a few ulps; with RADAR_FLAG_FP16, 1/32 relative).
 *           The environment variable RADAR_PEAKS_ONLY_FIRST_ROWS = R
 *           (1..64), a diagnostic, cuts the first listing to the R rows with
 *           the largest maxima; the result is the same.  Supported for N in
 *           {256, 512, 1024}, N' = 4N and 4 N_cp <= N, in every precision
 *           form (RADAR_E_UNSUPPORTED otherwise).
 * peaks:    output, k entries per frame at peaks + f*k; n_peaks[f] = number
 *           written (< k only if P has fewer than k local maxima).
 * status:   output, one word per frame (RADAR_ST_* bits; 0 = clean).
 * 1 <= k <= 64.
 * ------------------------------------------------------------------------ */
size_t radar_frame_workspace_size(const radar_frame_desc *d, int32_t n_frames, int32_t k);
int radar_frame_process(const radar_frame_desc *d, int32_t n_frames,
                        const radar_cf32 *Y, const radar_cf32 *A, int64_t frame_stride,
                        float *P, int64_t p_frame_stride,
                        int32_t k, radar_peak *peaks, int32_t *n_peaks, uint32_t *status,
                        void *ws, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * radar_frame_process_noalloc -- radar_frame_process for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same path, the same arguments and
 * results, minus the caller's workspace.
 *
 * The workspace is instead a library-owned device array of
 * RADAR_NOALLOC_WS_BYTES bytes, one per device, allocated when the library's
 * code is loaded on that device and held until the process ends; its address
 * is looked up once per device by radar_init.  Nothing is allocated or freed
 * by the call (no hipMalloc, no hipFree, no allocating library routine).
 * Limit: radar_frame_workspace_size(d, n_frames, k) must not exceed
 * RADAR_NOALLOC_WS_BYTES (one 1024 x 1024 frame with k = 8 needs about
 * 10.3 MiB, so up to three such frames per call); larger requests return
 * RADAR_E_WORKSPACE and enqueue nothing.
 * Every call on one device uses that device's one array, which keeps the
 * last call's contents: calls that overlap in time on one device (other
 * streams, other threads) race and give undefined results.  Successive calls
 * on one stream are fine; nothing in the array needs to start cleared.
 * Call radar_init once outside capture before capturing this call.
 * ------------------------------------------------------------------------ */
#define RADAR_NOALLOC_WS_BYTES (32u << 20)
int radar_frame_process_noalloc(const radar_frame_desc *d, int32_t n_frames,
                                const radar_cf32 *Y, const radar_cf32 *A, int64_t frame_stride,
                                float *P, int64_t p_frame_stride,
                                int32_t k, radar_peak *peaks, int32_t *n_peaks, uint32_t *status,
                                void *hip_stream);

/* ------------------------------------------------------------------------
 * radar_tap_wiener_weights -- per-tap LMMSE weights of the LMMSE-based DFT-CE
 * (Sec. III-A, Fig. 5), host only, no GPU call.
 *
 * With the tap estimate hhat(n) = h(n) + w(n) (the IDFT over the subcarriers
 * of the LS estimate, 1/N included), prior tap power p(n) = E|h(n)|^2 and
 * white noise of variance noise_var_tap per tap (sigma^2 mean(1/|a|^2) / N),
 * the least-mean-square linear estimate of h(n) is g(n) hhat(n) with
 *   g(n) = p(n) / (p(n) + noise_var_tap).
 * tap_power: host, n doubles >= 0; weights: host, n floats out.
 * RADAR_E_ARG on NULL pointers, n < 1, a negative or non-finite power, or
 * noise_var_tap < 0 or non-finite (noise_var_tap = 0 gives 1 where p > 0, 0
 * where p = 0).
 * ------------------------------------------------------------------------ */
int radar_tap_wiener_weights(const double *tap_power, int32_t n, double noise_var_tap, float *weights);

/* ------------------------------------------------------------------------
 * radar_periodogram -- Eq. 17 from a channel estimate the caller already has.
 *
 * H is an LS estimate (Eq. 16) laid out like Y.  If d->n_cp < N the DFT-CE of
 * Eq. 20-22 is applied first; d->zc_mode must be RADAR_ZC_NONE (H is already
 * de-precoded) and d->flags must not hold RADAR_FLAG_REFINE (no peaks, so
 * nothing to refine: RADAR_E_ARG otherwise); the precision flags apply.  P as for radar_frame_process.  The workspace size is
 * radar_frame_workspace_size(d, n_frames, 1).
 * ------------------------------------------------------------------------ */
int radar_periodogram(const radar_frame_desc *d, int32_t n_frames,
                      const radar_cf32 *H, int64_t frame_stride,
                      float *P, int64_t p_frame_stride,
                      void *ws, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * radar_detect_topk -- dominant peaks of given periodograms.
 *
 * P: n_frames float32 arrays [m_pad][n_pad] (frame f at P + f*p_frame_stride,
 * row m_pad/2 = Doppler 0).  Returns per frame the k largest 3x3 cyclic local
 * maxima, ranked by (value descending, flat index ascending), exactly as
 * radar_frame_process does.  m_pad, n_pad: powers of two in [4, 16384].
 * ------------------------------------------------------------------------ */
size_t radar_detect_workspace_size(int32_t m_pad, int32_t n_pad, int32_t n_frames, int32_t k);
int radar_detect_topk(const float *P, int32_t m_pad, int32_t n_pad, int32_t n_frames,
                      int64_t p_frame_stride, int32_t k,
                      radar_peak *peaks, int32_t *n_peaks,
                      void *ws, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * radar_fps_sft -- FPS-SFT, the sparse alternative to the periodogram
 * (Sec. III-C).
 *
 * Works on the LS estimate h[k, l] = y conj(z_k) / a of Eq. 16 at native
 * resolution (no DFT-CE, no window, no padding).  Of the descriptor only
 * n_sub (N), n_sym (M), zc_mode, zc_root, zc_shift and ld are used (N, M
 * in [16, 4096]; flags must be 0).  Q = lcm(N, M).  For N, M powers of two
 * Q = max(N, M) and the slices and their recovery stay in registers and LDS.
 * Otherwise (e.g. Table I's N = 2048, M = 560, Q = 71680) Q = P R with P the
 * power of two in Q and R odd; the Q-point DFT then runs as P-point and
 * R-point DFTs in the prime-factor mapping (no twiddles), and the recovery
 * keeps the spectra in global memory.  That path needs Q <= 131072,
 * P >= 16 and R <= 255 (RADAR_E_UNSUPPORTED otherwise), the ZC root
 * relatively prime to N (RADAR_E_NOT_COPRIME), and takes the ZC phase of
 * Eq. 23 for either parity of N.
 *
 * For each direction (alpha, beta) of s->dirs, in order, three slices
 * t -> h[(alpha t + tau1) mod N, (beta t + tau2) mod M], t < Q, at offsets
 * (tau1, tau2) = (0,0), (1,0), (0,1) are gathered and Q-point DFTed; their
 * bin m is the projection of the 2-D spectrum X = DFT_N x DFT_M of h onto
 * m = (alpha k1 Q/N + beta k2 Q/M) mod Q.  Recovery, per direction: subtract
 * the components found so far; visit bins by decreasing |S0|^2 (lower bin
 * first on ties) while |S0|^2 >= theta^2 = -ln(pfa) median(|S0|^2) / ln 2
 * and |S0|^2 > 1e-10 times the direction's largest raw |S0|^2; accept a bin
 * whose ratios S1/S0 and S2/S0 have magnitude within tol of 1 and whose
 * phases decode k1 = round(N arg(S1/S0) / 2 pi) mod N,
 * k2 = round(M arg(S2/S0) / 2 pi) mod M projecting back onto that bin; its
 * coefficient c = (N M / Q) S0 is added to a known (k1, k2) or starts a new
 * component.  Stops when k components are known or the directions run out.
 *
 * Output per frame: the n_peaks[f] <= k components as radar_peak entries in
 * periodogram coordinates, s = k2 wrapped to [-M/2, M/2), r = -k1 mod N,
 * p = |c|^2 / (N M) (the value of the native-resolution rectangular-window
 * periodogram of Eq. 17 at that cell for an isolated on-grid target), ranked
 * by (p descending, (s + M/2) N + r ascending); s_off = r_off = 0.
 * peaks: [n_frames][s->k]; status as for radar_frame_process, set from the
 * gathered samples only.
 * slices: optional output (NULL for none): the raw slice spectra
 *         [n_frames][n_dirs][3][Q] complex64 before any subtraction.
 * ws: device workspace of radar_fps_sft_workspace_size bytes.  With slices
 *     given and Q a power of two it may be NULL (the spectra live in slices);
 *     for other Q it is always needed (the DFT's first pass and the ZC table).
 * Errors: RADAR_E_ARG for bad pointers, n_frames outside [1, 65535], n_dirs
 * outside [1, 16], k outside [1, 64], pfa outside (0, 1), tol outside
 * (0, 1], a direction with alpha = 0 mod N and beta = 0 mod M, or flags != 0;
 * RADAR_E_UNSUPPORTED for N or M outside the sizes above;
 * RADAR_E_NOT_COPRIME as for radar_frame_process; RADAR_E_WORKSPACE.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_dirs;               /* I, number of slice directions, 1..16 */
  int32_t dirs[16][2];          /* (alpha, beta) per direction, any integers */
  int32_t k;                    /* components sought, 1..64 */
  float pfa;                    /* per-bin false-alarm probability (Table I: 1e-2) */
  float tol;                    /* 1-sparsity tolerance on |S1/S0|, |S2/S0| */
  int32_t flags;                /* must be 0 */
} radar_sft_desc;

/* Fills s with the default recovery settings: eight directions (1,1),
 * (1,-1), (1,2), (2,1), (1,-2), (2,-1), (1,0), (0,1), pfa = 1e-2, tol = 0.25,
 * and the given k. */
void radar_sft_default(radar_sft_desc *s, int32_t k);
size_t radar_fps_sft_workspace_size(const radar_frame_desc *d, const radar_sft_desc *s, int32_t n_frames);
int radar_fps_sft(const radar_frame_desc *d, const radar_sft_desc *s, int32_t n_frames,
                  const radar_cf32 *Y, const radar_cf32 *A, int64_t frame_stride,
                  radar_peak *peaks, int32_t *n_peaks, uint32_t *status,
                  radar_cf32 *slices, void *ws, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Batches of frames with uneven shapes -- the receive path of
 * radar_frame_process for many jobs at once, captured into one graph.
 *
 * A job is one frame with its own descriptor and its own buffers (device
 * pointers, caller-owned, laid out as for radar_frame_process with
 * n_frames = 1): Y, A [M][ld]; P [M'][N'] (16-byte aligned); peaks [k];
 * n_peaks and status one word each.  Descriptors follow radar_frame_process
 * (flags may hold RADAR_FLAG_REFINE and one precision flag).
 *
 * radar_batch_create groups the jobs by descriptor and k, uploads per-group
 * tables of the jobs' buffers into the workspace (synchronously), and builds
 * the launch sequence: per group the clear, taps, Doppler, range, peak (and
 * refinement) kernels, which address each frame through its table entry.
 * With RADAR_BATCH_TUNE it first times candidate launch plans per group on
 * the jobs' own data (persistent grid sizes; the four-phase or the
 * one-team-per-row range kernel) and keeps the fastest; choices are cached
 * per shape for the life of the process.  With RADAR_BATCH_GRAPH the whole
 * sequence is captured once into a HIP graph, and radar_batch_launch replays
 * it on the given stream; otherwise radar_batch_launch enqueues the kernels.
 * The plan keeps the job pointers and the workspace: both must stay valid
 * and unmoved until radar_batch_destroy.  Launches of one plan run in
 * stream order; a plan is not thread-safe.
 *
 * ws: device workspace of radar_batch_workspace_size bytes (the job tables
 *     plus every group's own scratch: the captured graph runs groups on up
 *     to four concurrent branches, heaviest groups first onto the least
 *     loaded branch).
 * Every job writes its periodogram: P must not be NULL here (the peaks-only
 * mode is radar_frame_process's).
 * Errors: as radar_frame_process per job (validation before any HIP call),
 * RADAR_E_ARG for n_jobs < 1, a NULL P, unknown batch flags or a NULL plan
 * pointer,
 * RADAR_E_HIP if a HIP call (upload, capture, instantiation) fails.
 * ------------------------------------------------------------------------ */
typedef struct {
  radar_frame_desc d;
  const radar_cf32 *Y, *A;
  float *P;
  radar_peak *peaks;
  int32_t *n_peaks;
  uint32_t *status;
  int32_t k;                    /* peaks sought, 1..64 */
} radar_frame_job;

enum { RADAR_BATCH_GRAPH = 1, RADAR_BATCH_TUNE = 2 };

typedef struct radar_batch radar_batch;
size_t radar_batch_workspace_size(const radar_frame_job *jobs, int32_t n_jobs);
int radar_batch_create(const radar_frame_job *jobs, int32_t n_jobs, int32_t flags, void *ws, size_t ws_bytes,
                       void *hip_stream, radar_batch **out);
int radar_batch_launch(radar_batch *b, void *hip_stream);
/* Number of shape groups, and the tuned plan of group g (k1_mult: taps
 * work-groups per CU, k3_mult: range work-groups per CU, k3_generic: 1 when
 * the one-team-per-row range kernel was chosen). */
int radar_batch_info(const radar_batch *b, int32_t g, int32_t *n_groups, int32_t *n_frames,
                     int32_t *k1_mult, int32_t *k3_mult, int32_t *k3_generic);
/* The rest of group g's tuned plan: k2_half_tile = 1 when the Doppler stage
 * runs tiles of half the taps, scan_groups = the peak scan's work-groups per
 * frame.  Outputs may be NULL.  RADAR_E_ARG for a NULL batch or g out of
 * range. */
int radar_batch_plan(const radar_batch *b, int32_t g, int32_t *k2_half_tile, int32_t *scan_groups);
void radar_batch_destroy(radar_batch *b);

/* ------------------------------------------------------------------------
 * The CNN sub-cell refiner (the learned alternative to RADAR_FLAG_REFINE;
 * the paper names machine learning as future work in Sec. V).
 *
 * Network: a 32 x 32 log-periodogram patch (rows Doppler, columns range,
 * centred on a detected cell) -> conv 3x3 1->32 -> conv 3x3 32->32 stride 2
 * -> conv 3x3 32->32 -> conv 3x3 32->32 stride 2 (zero padding 1, ReLU after
 * each) -> dense 2048->10 (ReLU) -> dense 10->2 = (range, Doppler) offset in
 * cells of the N' x M' grid.  theta: the radar_cnn_param_count() = 48576
 * FP32 parameters, in order conv1..conv4 (weights [co][ky][kx][ci], biases
 * [co]), dense1 (weights [10][2048] over the flattening (y*8+x)*32+c, biases
 * [10]), dense2 ([2][10], [2]).  The three 32->32 convolutions (forward and
 * input gradient) run on BF16 matrix cores with FP32 accumulation (weights
 * and activations rounded to BF16, gradients FP32); the rest is FP32.
 *
 * radar_cnn_patches: patch n = f*k + i of frame f's periodogram P
 *   (p_frame_stride floats apart, [m_pad][n_pad], powers of two >= 32) around
 *   peak i: ln(max(P, 1e-12 P_c)) - ln P_c over rows row-16..row+15 and
 *   columns r-16..r+15 (cyclic), P_c the peak cell; valid[n] = 1 if
 *   i < n_peaks[f] (else the patch is zero).  patches [n_frames*k][32][32].
 * radar_cnn_forward: out[b] = network(patches[b]), b < batch.
 * radar_cnn_gradient: grad = dL/dtheta and *loss = L (device pointers) for
 *   L = mean over the batch and both outputs of (network - labels)^2;
 *   labels [batch][2].
 * radar_cnn_adam: one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias
 *   correction for step >= 1) on theta with FP32 moments m, v.
 * radar_cnn_train_step: radar_cnn_gradient then radar_cnn_adam.
 * All arrays are device memory; ws is radar_cnn_workspace_size(batch, train)
 * bytes (train = 0 for forward only).  Errors: RADAR_E_ARG for NULL pointers
 * or batch outside [1, 65536], RADAR_E_UNSUPPORTED for grid sizes the patch
 * extraction does not support, RADAR_E_WORKSPACE.
 * ------------------------------------------------------------------------ */
int32_t radar_cnn_param_count(void);
size_t radar_cnn_workspace_size(int32_t batch, int32_t train);
int radar_cnn_patches(const float *P, int64_t p_frame_stride, int32_t m_pad, int32_t n_pad, int32_t n_frames,
                      int32_t k, const radar_peak *peaks, const int32_t *n_peaks, float *patches,
                      int32_t *valid, void *hip_stream);
int radar_cnn_forward(const float *theta, const float *patches, int32_t batch, float *out,
                      void *ws, size_t ws_bytes, void *hip_stream);
int radar_cnn_gradient(const float *theta, const float *patches, const float *labels, int32_t batch,
                       float *grad, float *loss, void *ws, size_t ws_bytes, void *hip_stream);
int radar_cnn_adam(float *theta, const float *grad, float *m, float *v, int32_t step, float lr,
                   void *hip_stream);
int radar_cnn_train_step(float *theta, float *m, float *v, int32_t step, float lr, const float *patches,
                         const float *labels, int32_t batch, float *loss, void *ws, size_t ws_bytes,
                         void *hip_stream);

/* ------------------------------------------------------------------------
 * radar_simulate_frames -- received frames from the time-domain model of
 * Sec. II-B.1 (Eq. 1-2 transmitter with cyclic prefix, Eq. 7-10 moving point
 * targets), to test how far Eq. 11's frequency-domain model holds.
 *
 * Time in samples T0 = 1/(N df); symbol l's useful part starts at
 * t_l = l (N + n_guard) + n_guard.  Target p has delay rho (samples = native
 * range bins), Doppler nu (bins of the M-point Doppler DFT) and amplitude b;
 * its CFO is eps = nu N / (M (N + n_guard)) subcarrier spacings and its
 * time-scale factor B = eps / fc_over_df, so its delay during symbol l is
 * d_l = rho + B t_l (held through the symbol).  While 0 <= d_l <= n_guard:
 *   Y[l][k'] = sum_m e^{-2 pi i k' m/N} sum_p b_p e^{+2 pi i nu_p (t_l + m)/(M (N + n_guard))}
 *              (1/N) sum_k A[l][k] e^{+2 pi i k (m - d_l)/N}      (+ noise[l][k'])
 * which keeps the inter-carrier interference (eps) and the range migration
 * (B) that Eq. 11 drops.  A delay outside [0, n_guard] sets RADAR_ST_ISI
 * in status[f] (the frame then lacks the inter-symbol interference).
 * A:        device, frame f at A + f*frame_stride, [M][ld] (the symbols on the
 *           subcarriers, after any precoding).
 * targets:  device, [n_frames][max_targets]; n_targets: device, [n_frames]
 *           (entries beyond n_targets[f] are ignored; clamped to [0, max]).
 * noise:    device, same layout as Y, added after the DFT, or NULL.
 * Y:        device output, same layout as A.  status: device, [n_frames]
 *           words ORed with RADAR_ST_ISI (not cleared), or NULL.
 * Sizes: N, M powers of two in [16, 4096]; 0 <= n_guard <= N; ld >= N;
 * 1 <= max_targets <= 1024; fc_over_df > 0 and finite.  No workspace.
 * ------------------------------------------------------------------------ */
typedef struct {
  float rho, nu;                /* delay (samples), Doppler (bins) */
  float b_re, b_im;             /* complex amplitude */
} radar_sim_target;

typedef struct {
  int32_t n_sub;                /* N */
  int32_t n_sym;                /* M */
  int32_t n_guard;              /* cyclic prefix in samples */
  int32_t max_targets;
  int64_t ld;
  double fc_over_df;            /* carrier over subcarrier spacing (Table I: 77e9 / 240e3) */
} radar_sim_desc;

int radar_simulate_frames(const radar_sim_desc *d, int32_t n_frames, const radar_cf32 *A, int64_t frame_stride,
                          const radar_sim_target *targets, const int32_t *n_targets,
                          const radar_cf32 *noise, radar_cf32 *Y, uint32_t *status, void *hip_stream);

/* ------------------------------------------------------------------------
 * radar_papr -- peak-to-average power ratio of Eq. 25 per OFDM symbol.
 *
 * papr[f*M + l] = max_n |x_n|^2 / mean_n |x_n|^2 (linear) with x the N-point
 * IDFT of symbol l of frame f (the transmitted samples at the Nyquist rate;
 * the cyclic prefix repeats samples and leaves the ratio unchanged), 0 for
 * an all-zero symbol.  A: device, frame f at A + f*frame_stride, [M][ld], the
 * symbols on the subcarriers after any precoding; papr: device [n_frames][M].
 * N, M powers of two in [16, 4096]; ld >= N.  No workspace.
 * ------------------------------------------------------------------------ */
int radar_papr(int32_t n_sub, int32_t n_sym, int64_t ld, int32_t n_frames, const radar_cf32 *A,
               int64_t frame_stride, float *papr, void *hip_stream);

/* ------------------------------------------------------------------------
 * radar_hpa -- the high power amplifier of Eq. 26 on every symbol's
 * transmitted samples, returned as subcarrier symbols.
 *
 * Per symbol: x = IDFT_N(A) (the samples; the prefix repeats them), then the
 * amplitude-only soft limiter |x'| = |x| / sqrt(1 + (|x| / (xbar 10^{q/10}))^2)
 * with xbar the mean of |x_n| over the symbol, the phase kept, and
 * out = DFT_N(x').  Feed out to radar_simulate_frames as the transmitted
 * symbols while the radar still divides by A.  An all-zero symbol stays zero.
 * A, out: device, frame f at + f*frame_stride, [M][ld]; out may equal A.
 * q_db: the state level (2 in Sec. III-B), finite.  N, M powers of two in
 * [16, 4096]; ld >= N.  No workspace.
 * ------------------------------------------------------------------------ */
int radar_hpa(int32_t n_sub, int32_t n_sym, int64_t ld, int32_t n_frames, const radar_cf32 *A,
              int64_t frame_stride, double q_db, radar_cf32 *out, void *hip_stream);

/* ------------------------------------------------------------------------
 * Stage timing -- a profiling aid, off by default.
 *
 * radar_timing_start(max_launches) creates HIP events for up to max_launches
 * launches of each stage; until radar_timing_stop, every stage launch of the
 * calls above records an event pair on its own stream around the kernel(s)
 * of that stage.  radar_timing_stop waits for the recorded events, writes per
 * stage the summed kernel time in milliseconds and the number of launches
 * timed (arrays of RADAR_NUM_STAGES entries), and destroys the events.
 * Launches beyond max_launches are not timed.  Not thread-safe: time one
 * stream at a time.
 * ------------------------------------------------------------------------ */
enum {
  RADAR_STAGE_TAPS = 0,         /* de-precode, divide, IDFT_N, truncate   (Eq. 16, 20-21) */
  RADAR_STAGE_DOPPLER = 1,      /* M'-point Doppler DFT of the taps       (Eq. 17) */
  RADAR_STAGE_RANGE = 2,        /* DFT_N back, window, N'-point range DFT, |.|^2 (Eq. 22, 17) */
  RADAR_STAGE_PEAKS = 3,        /* local maxima and top-k */
  RADAR_STAGE_REFINE = 4,       /* sub-cell refinement (RADAR_FLAG_REFINE) */
  RADAR_STAGE_SFT_SLICES = 5,   /* FPS-SFT slice gather and Q-point DFTs */
  RADAR_STAGE_SFT_DECODE = 6,   /* FPS-SFT recovery */
  RADAR_NUM_STAGES = 7
};
int radar_timing_start(int32_t max_launches);
int radar_timing_stop(double *ms_total, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* RADAR_H */
