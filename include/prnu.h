/*
 * prnu.h -- C ABI of the MI355X (gfx950) EIS-inversion grid search.
 *
 * Method (arXiv 2207.14507, "GPU-accelerated SIFT-aided source identification of
 * stabilized videos"):
 *   - A frame residual W is tested against a camera fingerprint K by the
 *     Peak-to-Correlation Energy of Eq. (3), built on the normalised
 *     cross-correlation of Eq. (1).
 *   - Electronic stabilisation is modelled by the projective map of Eq. (4); the
 *     search of Sec. 3.2 (operator CORRECTION) restricts it to a similarity:
 *     t11 = t22 = s cos(theta), t12 = -t21 = s sin(theta), t31 = t32 = 0, with
 *     theta in degrees.
 *   - For every candidate (s, theta) of a grid, the residual is inverse-warped
 *     (bilinear, taps outside the image are zero) about the image centre.  It is
 *     then correlated with K at every circular shift, and the PCE is taken with
 *     the signed peak searched within +-shift_radius and an 11x11 cyclic
 *     exclusion neighbourhood.  The candidate of maximum PCE is kept (ties: the
 *     lowest candidate index, scale-major then rotation).
 *   - Consecutive frames are chained (Algorithm 1): with warm start, a frame
 *     searches a local grid centred on the previous frame's estimate (T_init of
 *     Sec. 3.2).  It falls back to the full grid when the local best PCE is below
 *     a threshold.
 *   - The video decision thresholds the mean of the per-frame maxima gamma
 *     (Sec. 3.2, last paragraph).
 *
 * Conventions
 *   - Images are row-major, height = M rows, width = N columns; strides in elements.
 *   - Sizes: the fingerprint's M and N must be lengths the library is built for
 *     (see prnu_supported_lengths); N must be even.  Frames are M x N, or smaller
 *     (M' x N' with M' <= M, N' <= N; Sec. 2 zero-pads the smaller operand of
 *     Eq. (1)): a smaller frame is inverse-warped about its own centre, placed at
 *     rows 0..M'-1, columns 0..N'-1 of an M x N array of zeros, and the peak is
 *     searched over -R <= dy <= M - M' + R, -R <= dx <= N - N' + R (R =
 *     shift_radius): the linear shifts 0 <= delta <= (M - M', N - N') of Eq. (3)
 *     widened by R.  (dx, dy) is then the frame's position inside the fingerprint.
 *     Frames need M', N' >= 2*shift_radius + 11.  Otherwise PRNU_E_SHAPE, also for
 *     a frame larger than the fingerprint.
 *   - Ownership: the caller owns every buffer it passes; the library copies what
 *     it keeps.  Device pointers (on_device = 1) are read on the caller's stream
 *     (a hipStream_t, NULL = default stream), and must stay alive until the call
 *     returns (prnu_search_frames) or until prnu_submit_video returns (submit
 *     copies the frames).
 *   - Errors: functions return a negative prnu_status; no exception crosses the
 *     ABI.  prnu_last_error() gives a human-readable detail for the calling
 *     thread.  A HIP runtime failure marks the context as failed: every later
 *     call on it returns PRNU_E_DEVICE.
 *   - Threading: all calls on one context are thread-safe.
 *   - Test hook: the environment variable PRNU_FAULT, read by prnu_create, takes a
 *     comma-separated list of "launch:N" and "stage:N".  The Nth launch of search
 *     kernels (or the Nth frame staging) on that context then fails the way a HIP
 *     failure does (PRNU_E_DEVICE, the context marked failed, every video in the
 *     serving engine ended with PRNU_E_DEVICE) before any of its work is issued.
 */
#ifndef PRNU_H_
#define PRNU_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PRNU_OK = 0,
  PRNU_PENDING = 1,      /* prnu_poll: the video is not finished yet */
  PRNU_E_ARG = -1,       /* invalid argument (null pointer, bad option value) */
  PRNU_E_SHAPE = -2,     /* unsupported or mismatched image size */
  PRNU_E_NOMEM = -3,     /* allocation failed or the request exceeds the HBM budget */
  PRNU_E_DEVICE = -4,    /* HIP runtime error; the context is unusable */
  PRNU_E_HANDLE = -5,    /* unknown fingerprint handle or ticket */
  PRNU_E_BUSY = -6,      /* submission queue full: retry later */
  PRNU_E_NONFINITE = -7, /* input holds NaN or Inf */
  PRNU_E_CANCELLED = -8  /* the video was cancelled */
} prnu_status;

typedef enum { PRNU_F32 = 0, PRNU_BF16 = 1 } prnu_dtype;

typedef struct prnu_ctx prnu_ctx; /* opaque */
typedef uint64_t prnu_fp;         /* fingerprint handle, 0 is never valid */
typedef uint64_t prnu_ticket;     /* submitted-video handle, 0 is never valid */

typedef struct {
  int32_t device;            /* HIP device ordinal */
  uint64_t hbm_budget_bytes; /* device memory the serving engine may hold for videos (0 = 16 GiB) */
  int32_t max_slots;         /* videos admitted concurrently by the serving engine (0 = 16) */
  const char* tune_cache_path; /* autotuner cache file (NULL = none): read at create, rewritten
                                  whenever a shape is tuned */
  uint32_t flags;            /* PRNU_FLAG_* below, or 0 */
} prnu_config;

/* Every launch set of the search kernels (warp + row DFT, column DFT + product, band
 * inverse, PCE; one set per FFT batch of candidates) is captured once into a HIP graph
 * per distinct shape, candidate count and buffer set, and replayed afterwards. */
#define PRNU_FLAG_NO_GRAPHS 1u
/* The launch schedule of a shape is picked by timing the candidates on first use
 * (see prnu_tune); with this flag the memory-bound default is used instead. */
#define PRNU_FLAG_NO_AUTOTUNE 2u

/* A uniform grid of n nodes over [lo, hi], generated as centre + k*step (k centred). */
typedef struct {
  int32_t n_scale;
  double scale_lo, scale_hi;
  int32_t n_rot;
  double rot_lo_deg, rot_hi_deg;
} prnu_grid;

typedef struct {
  prnu_grid full;              /* the exhaustive grid (e.g. 41 x 21 over [0.85,1.15] x [-2,2] deg) */
  int32_t shift_radius;        /* peak searched over |dy|, |dx| <= shift_radius (equal sizes) */
  int32_t exclusion;           /* side of the exclusion neighbourhood; must be 11 (Eq. 3) */
  int32_t warm;                /* 0: every frame on the full grid; 1: warm start */
  int32_t local_n_scale, local_n_rot; /* local grid size (e.g. 9 x 9) */
  double local_dscale, local_drot_deg;/* local grid steps (e.g. 0.005, 0.1 deg) */
  double fallback_pce;         /* local best below this also searches the full grid (e.g. 60) */
  int32_t has_init;            /* warm start of the first frame from (init_scale, init_rot_deg) */
  double init_scale, init_rot_deg;
  double tau;                  /* decision threshold on mean gamma (the paper's operating point: 19.5) */
  /* The paper's own coarse-to-fine schedule of CORRECTION (Sec. 3.2, Eq. (8)) instead of
   * the fixed grid (refine = 1; requires warm = 0; the full grid is then unused).
   * Iteration n searches every pair (lambda, theta) with lambda = lambda^(n-1) +
   * alpha * refine_scale_step * 10^-(n-1) and theta = theta^(n-1) + alpha *
   * refine_rot_step * 10^-(n-1), integer |alpha| <= refine_half; iteration 1 uses the
   * dense absolute rotation grid refine_rot_lo_deg, + refine_rot_step, ...,
   * refine_rot_hi_deg instead.  (lambda^(0), theta^(0)) = (1, 0), or the initial
   * transform when has_init.  Stops when an iteration's estimate equals the previous one
   * or after refine_max_iter iterations; gamma is the largest PCE evaluated.  The
   * paper's values: half 5, 3 iterations, steps 0.01 and 0.1 deg, range [-5, 5] deg. */
  int32_t refine;
  int32_t refine_half;
  int32_t refine_max_iter;
  double refine_scale_step;
  double refine_rot_step;
  double refine_rot_lo_deg, refine_rot_hi_deg;
} prnu_search_opts;

/* n_frames residual frames of one video.  BF16 frames carry one float32 scale per
 * frame: the residual is frame_scale[f] * bf16 value.  n_frames may be 0 (data and
 * frame_scale may then be NULL): the searches return no results and a summary of 0
 * frames with mean PCE 0 and decision 0, a video is done at submission, and
 * prnu_extract_residuals does nothing. */
typedef struct {
  const void* data;
  prnu_dtype dtype;
  const float* frame_scale; /* BF16 only; host array when on_device = 0, else device */
  int32_t n_frames, height, width;
  int64_t frame_stride, row_stride; /* elements */
  int32_t on_device;
  void* stream; /* hipStream_t the device data is ordered on (on_device = 1); the library's
                   reads wait for the work queued on it before the call.  NULL is the
                   legacy default stream (torch's default stream). */
} prnu_frames;

typedef struct {
  double pce;        /* gamma of the frame: maximum PCE over the searched candidates */
  double rho;        /* NCC of Eq. (1) at the peak */
  double scale, rot_deg; /* winning candidate */
  int32_t dx, dy;    /* peak shift: the frame content sits at p + (dx, dy) of the fingerprint */
  int32_t cand_index;/* index of the winner in the evaluated list (local grid first, then full;
                        with refine, the iterations' grids in order) */
  int32_t fell_back; /* warm start fell back to the full grid */
  int32_t n_evaluated;
  int32_t status;    /* prnu_status of this frame */
  int32_t iterations;/* refinement iterations run (refine = 1), else 0 */
  int32_t used_init; /* prnu_search_with_transform: the caller's transform scored higher
                        than the frame as is and seeded the refinement */
} prnu_frame_result;

typedef struct {
  double mean_pce;   /* mean of gamma over the frames */
  int32_t decision;  /* mean_pce > tau */
  int32_t n_frames;
  double queue_s;    /* submit -> admission */
  double latency_s;  /* submit -> completion */
} prnu_video_summary;

/* Context: one per device. */
prnu_status prnu_create(const prnu_config* cfg, prnu_ctx** out);
void prnu_destroy(prnu_ctx* ctx);
const char* prnu_status_string(prnu_status s);
const char* prnu_last_error(void);

/* Lengths (rows or columns) the kernels are built for; returns the count and writes
 * at most cap of them. */
int32_t prnu_supported_lengths(int32_t* out, int32_t cap);

/* Eq. (1)-(3) preparation of a fingerprint (once per fingerprint):
 *  - mean and norm of K in FP64;
 *  - K - mean;
 *  - its 2-D DFT, stored device-resident with the DC bin forced to zero.
 * K is M x N float32 with row_stride elements per row, host (on_device = 0) or device
 * memory ordered on stream (NULL: the legacy default stream).  The library copies what
 * it needs; *out receives a handle. */
prnu_status prnu_open_fingerprint(prnu_ctx* ctx, const float* K, int32_t height, int32_t width,
                                  int64_t row_stride, int32_t on_device, void* stream, prnu_fp* out);
prnu_status prnu_close_fingerprint(prnu_ctx* ctx, prnu_fp fp);

/* The grid search of Sec. 3.2 on every frame of one video against fingerprint fp
 * (synchronous).  out has frames->n_frames entries; summary (optional) receives the
 * video decision.  The plain form (opts->warm = 0) searches the full grid on every
 * frame; the warm form chains the frames as described above. */
prnu_status prnu_search_frames(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames,
                               const prnu_search_opts* opts, prnu_frame_result* out,
                               prnu_video_summary* summary);

/* Per-candidate scores of one frame (the exhaustive step without the argmax): PCE,
 * NCC and peak shift of every candidate of the full grid, scale-major order.  Arrays
 * have n_scale * n_rot entries.  PRNU_E_ARG if frame is not in [0, n_frames). */
prnu_status prnu_score_grid(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames, int32_t frame,
                            const prnu_search_opts* opts, double* pce, double* rho,
                            int32_t* dx, int32_t* dy);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): prnu_score_grid with every buffer on the device and
 * no allocation of any kind.  frames must be device memory (on_device = 1; for bf16,
 * frame_scale a device array too); pce (required), rho, dx and dy are device arrays of
 * n_scale * n_rot entries.  The work is queued on frames->stream (NULL: the legacy
 * default stream) and the call returns without waiting: the outputs are valid once that
 * stream has run it.  Intermediate data live in a fixed 128 MiB device array of the
 * library (one per device, held until the process ends), shared by every call on that
 * device: calls that overlap on one device (from any thread or context, on any streams)
 * race and must not be issued.  Limits: at most 65536 candidates, and the zero-bordered
 * frame, the candidate lists and one candidate's workspace must fit the array (every
 * shape the library supports does).  The fingerprint's transform tables exist once
 * prnu_open_fingerprint has returned.  Errors: as prnu_score_grid, plus PRNU_E_ARG for
 * host frames or too many candidates and PRNU_E_NOMEM when the scratch array is too
 * small; nothing is queued then. */
prnu_status prnu_score_grid_noalloc(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames, int32_t frame,
                                    const prnu_search_opts* opts, double* pce, double* rho, int32_t* dx,
                                    int32_t* dy);

/* The noise residuals W(I) = I - F(I) of Sec. 2 (defined before Eq. (2)), F being the
 * wavelet denoiser the paper cites, in the form PRNU work applies it:
 *   - a 4-level periodic orthonormal 2-D wavelet transform with the 8-tap Daubechies
 *     filter (4 vanishing moments, minimum phase);
 *   - per detail coefficient c, the signal variance v = max(0, m - sigma0^2), m the
 *     smallest of the means of c^2 over the 3x3, 5x5, 7x7 and 9x9 windows around it
 *     (zero outside the subband);
 *   - the residual keeps c sigma0^2 / (v + sigma0^2) of every detail coefficient (what
 *     the Wiener estimate c v / (v + sigma0^2) removes) and none of the coarsest
 *     approximation, transformed back.
 * Sides that are not multiples of 16 are extended by mirroring the last rows and
 * columns (the edge itself not repeated) and the residual is cropped back.  sigma0 is
 * the noise standard deviation in the images' units (3 for intensities in [0, 255]);
 * sigma0 = 0 gives zero residuals.
 * images: n_frames float32 images of height x width >= 9 x 9 (any strides, host or
 * device memory; device memory is read after the work queued on images->stream).
 * out: n_frames * height * width floats, tight row-major, in host memory or
 * (out_on_device = 1) device memory.  Synchronous.  Errors: PRNU_E_ARG (null pointers,
 * dtype not float32, negative or non-finite sigma0, strides), PRNU_E_SHAPE (fewer than
 * 9 rows or columns), PRNU_E_NOMEM. */
prnu_status prnu_extract_residuals(prnu_ctx* ctx, const prnu_frames* images, double sigma0, float* out,
                                   int32_t out_on_device);

/* Eq. (2): the reference fingerprint K = (sum_l I_l W_l) / (sum_l I_l I_l), pixel-wise,
 * from L float32 images and their noise residuals W_l = I_l - F(I_l) (from
 * prnu_extract_residuals or the caller's own denoiser F; same count and size; host or
 * device memory, each ordered on its own stream when on the device).  Accumulated in
 * FP64; 0 where every image is 0.  K receives height x width floats, row-major, in host
 * memory or (out_on_device = 1, 16-byte aligned) device memory; synchronous.  The result
 * can be passed to prnu_open_fingerprint.  Errors: PRNU_E_ARG (null pointers, no images,
 * dtype not float32, strides), PRNU_E_SHAPE (counts or sizes differ), PRNU_E_NOMEM. */
prnu_status prnu_estimate_fingerprint(prnu_ctx* ctx, const prnu_frames* images, const prnu_frames* residuals,
                                      float* K, int32_t out_on_device);

/* Eq. (4) in its general 8-parameter form: PCE, NCC and peak shift of n arbitrary
 * transforms T on one frame.  T holds n row-major 3 x 3 matrices in centred
 * coordinates (origin at the image centre ((N-1)/2, (M-1)/2)), mapping stabilised to
 * original coordinates as in Eq. (4); the frame is resampled at
 * pi(T^-1 (q - c, 1)) + c, pi(X, Y, Z) = (X/Z, Y/Z), bilinear, zero outside the image
 * and beyond the horizon (Z <= 0).  The similarity candidate (s, theta) is
 * [[s cos, s sin, 0], [-s sin, s cos, 0], [0, 0, 1]].  PRNU_E_ARG for a non-finite or
 * singular T. */
prnu_status prnu_score_transforms(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames, int32_t frame,
                                  const double* T, int32_t n, int32_t shift_radius, double* pce, double* rho,
                                  int32_t* dx, int32_t* dy);

/* Algorithm 1's co-registration branch with the homography supplied by the caller: for
 * each frame f, H[f] (row-major 3 x 3, conventions as above) is scored against the frame
 * as is; where it scores higher, the refinement (opts->refine must be 1) starts from the
 * scale and rotation nearest to H[f] (theta = atan2(t12 - t21, t11 + t22),
 * s = sqrt|t11 t22 - t12 t21|), otherwise from (1, 0) or opts' initial transform.
 * out[f].used_init records the choice. */
prnu_status prnu_search_with_transform(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames,
                                       const prnu_search_opts* opts, const double* H, prnu_frame_result* out,
                                       prnu_video_summary* summary);

/* Serving: continuous batching of videos against device-resident fingerprints.
 * submit copies the frames into library-owned memory, so the caller may free them
 * on return; it returns PRNU_E_BUSY when the submission queue is full.  Videos are
 * admitted while slots and the HBM budget allow; PRNU_E_NOMEM if one video alone
 * exceeds the budget.  poll returns PRNU_PENDING until the video is done, then its
 * status exactly once (results copied to out[n_frames] and *summary when non-NULL),
 * after which the ticket is retired (PRNU_E_HANDLE).  timeout_ms < 0 waits forever. */
prnu_status prnu_submit_video(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames,
                              const prnu_search_opts* opts, prnu_ticket* out);
prnu_status prnu_poll(prnu_ctx* ctx, prnu_ticket t, int32_t timeout_ms, prnu_frame_result* out,
                      prnu_video_summary* summary);
prnu_status prnu_cancel(prnu_ctx* ctx, prnu_ticket t);

/* Launch schedule of the search for frames of height x width, shift radius and dtype:
 * the FFT batch (candidates per launch set) and the block order of the row and column
 * kernels (0: candidates fastest, so blocks in flight together share frame rows and
 * fingerprint strips in cache; 1: a candidate's tiles together).  Unless the context
 * was created with PRNU_FLAG_NO_AUTOTUNE, a shape not yet tuned (in this context or
 * its cache file) is tuned now: every schedule whose workspace fits the tuner's memory
 * cap runs on zero-valued synthetic data (the kernels' time does not depend on the
 * values) and the fastest per candidate is kept, stored in the cache file if one is
 * set.  Cache lines that do not parse, or hold a batch below 1 or above 4096 or an
 * unknown order, are skipped; a cached batch whose workspace exceeds the memory cap is
 * halved until it fits (results never depend on the batch).  Outputs may be NULL;
 * *ns_per_candidate is the measured time (0 if untuned), *from_cache is 1 if the
 * schedule was read from the cache file. */
prnu_status prnu_tune(prnu_ctx* ctx, int32_t height, int32_t width, int32_t shift_radius, prnu_dtype dtype,
                      int32_t* batch, int32_t* order, double* ns_per_candidate, int32_t* from_cache);

/* Graphs captured and replayed so far by the synchronous search of this context. */
prnu_status prnu_graph_stats(prnu_ctx* ctx, int64_t* captures, int64_t* replays);

/* Host-side helpers (no device needed).
 * prnu_candidates writes the (scale, rotation) pairs of one candidate grid, scale-major,
 * as out[2 i], out[2 i + 1], and returns their count (writing at most cap pairs; a
 * negative status on bad arguments): kind 0 the full grid of opts, kind 1 the local
 * warm-start grid around (cs, ct), kind 2 refinement iteration `iteration` (1-based)
 * around (cs, ct).  prnu_check_opts returns the status a search would return for opts
 * alone (PRNU_OK or PRNU_E_ARG with prnu_last_error set). */
int32_t prnu_candidates(const prnu_search_opts* opts, int32_t kind, int32_t iteration, double cs, double ct,
                        double* out, int32_t cap);
prnu_status prnu_check_opts(const prnu_search_opts* opts);

/* Kernel timing with HIP events on the library's stream (for roofline reports).
 * enable != 0 starts recording and clears the counters; read writes, per kernel
 * family (warp+row FFT, column FFT+product, band row inverse, PCE), launches, total
 * milliseconds, candidates processed and the algorithmic bytes moved. */
#define PRNU_NUM_KERNELS 4
typedef struct {
  const char* name;
  int64_t launches;
  double total_ms;
  int64_t candidates;
  double algo_bytes;
} prnu_kernel_stats;
prnu_status prnu_profile_enable(prnu_ctx* ctx, int32_t enable);
prnu_status prnu_profile_read(prnu_ctx* ctx, prnu_kernel_stats* out /* [PRNU_NUM_KERNELS] */);

#ifdef __cplusplus
}
#endif
#endif /* PRNU_H_ */
