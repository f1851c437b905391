/*
 * cdmd.h -- C ABI of the MI355X compressed-DMD (cDMD) background-modeling library.
 *
 * The calls follow the problem statement of Erichson, Brunton and Kutz,
 * "Compressed Dynamic Mode Decomposition for Background Modeling":
 *
 *   cdmd_create      the parameters of Algorithm 1 (target rank k, samples p) and the
 *                    choice of measurement matrix C (Section 3.3); draws/prepares C.
 *   cdmd_fit         Algorithm 1 through the amplitudes: sketch Y = C X, Y' = C X'
 *                    (eq. (eq:YCX)), truncated SVD of Y, A~ = U* Y' V S^-1, eig(A~),
 *                    full modes Phi = X' V S^-1 W (eq. (Eq:cDMDModes)) and amplitudes
 *                    b = lstsq(Phi, x_1) (eq. (eq:b)).
 *   cdmd_modes       returns Lambda, b, the singular values, and optionally Phi.
 *   cdmd_select      background-mode selection: sparsity-constrained amplitudes by
 *                    orthogonal matching pursuit (Section 2.3, eq. (eq:sparsecoding)),
 *                    the zero mode or an |omega| threshold (Section 2.2), or an explicit
 *                    support.
 *   cdmd_background  L = Re(Phi_S diag(beta) V_S) (Section 2.2, eq. (equ:DMDTerms)) or
 *                    the static model Re(Phi_S beta) (Section 2.3).
 *   cdmd_foreground  mask = |x_jt - L_jt| > tau (Section 4, eq. (eq:thres)).
 *
 * Conventions
 *   Video layout: frame-major.  Frame t (0-based) of a video starts at element t*ld;
 *     pixel i of that frame is element t*ld + i.  ld >= n.  uint8 pixels are read as
 *     u/255; float32 pixels as they are.  The paper's X is pixels x frames, the
 *     transpose of this layout.
 *   Device pointers ("d_" prefix) are device memory of the current HIP device; host
 *     pointers ("h_" prefix, or plain arrays) are host memory.  All pointers are
 *     borrowed for the duration of the call only; the library keeps no reference.
 *   Streams: `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work of a call is enqueued on it.  Calls that return host results
 *     synchronise the stream before returning.
 *   Errors: every call returns a cdmd_status; arguments are validated before any
 *     device work.  cdmd_last_error() gives a thread-local message for the last
 *     failing call on the calling thread.  No call aborts or throws.
 *   Thread safety: one model must not be used by two threads at once; distinct models
 *     are independent.
 *   Determinism: the same inputs, configuration and seed give bitwise-identical
 *     results on the same device.
 */
#ifndef CDMD_H
#define CDMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CDMD_ABI_VERSION 1

typedef enum {
  CDMD_OK = 0,
  CDMD_E_INVALID_ARG = 1,     /* argument or configuration out of range */
  CDMD_E_UNSUPPORTED = 2,     /* valid request the library does not implement */
  CDMD_E_OUT_OF_MEMORY = 3,   /* device or host allocation failed */
  CDMD_E_DEVICE = 4,          /* HIP runtime error, or no usable gfx950 device */
  CDMD_E_RANK_DEFICIENT = 5,  /* sigma_k <= 1e-6 sigma_1: the rank-k SVD is undefined */
  CDMD_E_NUMERIC = 6,         /* NaN/Inf, eigensolver failure, |lambda|^(m-1) > 1e30 */
  CDMD_E_STATE = 7            /* call order violated (e.g. foreground before select) */
} cdmd_status;

typedef enum { CDMD_U8 = 0, CDMD_F32 = 1 } cdmd_dtype;

/* Measurement matrix C (p x n), Section 3.3 */
typedef enum {
  CDMD_SKETCH_GAUSSIAN = 0,   /* i.i.d. N(0, 1/p); entry (r, j) is a pure function of
                                 (seed, r, j): Philox4x32-10 counter (j>>2, r, 0, 0),
                                 key (seed lo, seed hi), Box-Muller on output words
                                 (w0,w1) -> pixels 4(j>>2)+0,1 and (w2,w3) -> +2,3,
                                 uniforms (w+1) 2^-32; never stored */
  CDMD_SKETCH_SPARSE = 1,     /* each row holds nnz entries +/-1 at distinct pixels,
                                 given by the caller's index/sign table */
  CDMD_SKETCH_SPIXEL = 2,     /* single-pixel C = R: p distinct pixels, weight +1
                                 (nnz = 1), given by the caller's index table */
  CDMD_SKETCH_SRFT = 3        /* subsampled randomised Fourier transform C = R F D / sqrt(p):
                                 D diagonal with entries exp(2 pi i u_j), u_j = word j mod 4
                                 of Philox4x32-10 on the counter (j>>2, 0, 0, 1) with the
                                 key of the Gaussian C, times 2^-32; F the unnormalised n-point
                                 DFT, F(f, j) = exp(-2 pi i f j / n); R keeps the p distinct
                                 DFT rows f given in sparse_idx (nnz = 1, weights +1).  The
                                 sketch is complex: FP32 form only, the small linear algebra
                                 complex on the host; no batches */
} cdmd_sketch;

/* Arithmetic of the sketch and of the mode lift / reconstruction passes.  The
   SVD, eigensolves and amplitude solves are always float64. */
typedef enum {
  CDMD_PREC_FP32 = 0,   /* float32 products, float32 accumulation per tile, float64
                           across tiles */
  CDMD_PREC_BF16 = 1,   /* bfloat16 operands (RNE), float32 accumulation (MFMA) */
  CDMD_PREC_FP8 = 2     /* OCP e4m3fn operands (RNE, saturating), float32
                           accumulation (MFMA); sketch only */
} cdmd_prec;

/* Modes the amplitudes b and the selection are computed on. */
typedef enum {
  CDMD_AMP_FULL = 0,       /* the full modes Phi = X' V S^-1 W and x_1 (eq. (eq:b)) */
  CDMD_AMP_COMPRESSED = 1  /* the compressed modes Phi_Y = Y' V S^-1 W and the first
                              compressed frame y_1 (Remark 3, Section 3.2) */
} cdmd_amp_space;

typedef enum {
  CDMD_SEL_OMP = 0,        /* orthogonal matching pursuit with K atoms on x_1 */
  CDMD_SEL_ZERO_MODE = 1,  /* the mode with the smallest |log lambda| */
  CDMD_SEL_OMEGA = 2,      /* all modes with |log lambda| < omega_thr */
  CDMD_SEL_EXPLICIT = 3,   /* caller-given support; beta refitted by least squares */
  CDMD_SEL_ALL = 4         /* every mode, beta = b */
} cdmd_selector;

typedef struct {
  int64_t n;            /* pixels per frame, n >= m */
  int64_t m;            /* frames, m >= 2 */
  int64_t ld;           /* elements between frame starts, ld >= n */
  int32_t k;            /* target rank, 1 <= k <= min(p, m-1) */
  int32_t p;            /* sketch rows (samples), p >= k */
  int32_t nnz;          /* nonzeros per row of a sparse C (1..32); 1 for single-pixel */
  int32_t dtype;        /* cdmd_dtype of the video */
  int32_t sketch;       /* cdmd_sketch */
  int32_t sketch_prec;  /* cdmd_prec of the sketch (sparse/single-pixel: exact integer
                           sums for uint8 video, float64 for float32 video) */
  int32_t lift_prec;    /* cdmd_prec of the lift and reconstruction (FP32 or BF16) */
  uint64_t seed;        /* Gaussian C */
  const int32_t* sparse_idx;  /* host, p*nnz row-major pixel indices in [0, n),
                                 distinct within a row (single-pixel: distinct over
                                 all rows); required for SPARSE and SPIXEL.  SPARSE
                                 only: -1 marks an empty slot, so rows may hold fewer
                                 than nnz nonzeros (the i.i.d. very sparse C of Section
                                 3.3); at least one slot must be used */
  const int8_t* sparse_sign;  /* host, p*nnz entries +1/-1 (NULL = all +1) */
} cdmd_config;

/* Opaque, library-owned model: the prepared C, device workspace sized for the
   configuration, and the results of the last fit (Lambda, W, G = V S^-1 W,
   H = Phi^H Phi, c = Phi^H x_1, b, the selection). */
typedef struct cdmd_model cdmd_model;

typedef struct {
  int32_t fitted;            /* 1 after a successful cdmd_fit */
  int32_t selected;          /* 1 after a successful cdmd_select */
  int32_t warn_few_samples;  /* 1 if p < k ln(n/k) (Section 4 guidance), else 0 */
  int32_t n_selected;        /* |S| */
  double sigma_ratio;        /* sigma_k / sigma_1 of the last fit */
  double x1_norm2;           /* ||x_1||^2 */
  double omp_residual2;      /* ||x_1 - Phi_S beta||^2 after selection */
  double ms_sketch;          /* host wall time of the last fit: sketch + Gram + copy */
  double ms_small_la;        /* ... float64 SVD / eigensolves on the host */
  double ms_lift;            /* ... lift + reduction + copy */
  double ms_host_post;       /* ... amplitudes and canonical order */
  int32_t lanczos_steps;     /* Krylov dimension used by the symmetric eigensolver */
  int32_t timing;            /* 1 if kernel timing is enabled (cdmd_set_timing) */
  /* Device time (ms, HIP events on the call's stream) of the last launch of each
     kernel group, valid when timing is enabled: sketch (incl. slot reduction), Gram,
     lift (incl. partial reduction), reconstruction/threshold. */
  double gpu_ms_sketch, gpu_ms_gram, gpu_ms_lift, gpu_ms_recon;
  int32_t lift_grid;         /* lift workgroups in use (cdmd_autotune may change it) */
  int32_t sketch_slices;     /* pixel slices of the dense Gaussian sketch (0 otherwise) */
  int32_t sparse_form;       /* after cdmd_autotune: uint8 sparse sketch form, -1 gather
                                (byte loads per triple), 10 F + V streaming (F frames per
                                group, V 16-byte vectors per thread); 0 not tuned */
  double gpu_ms_lanczos;     /* device small LA, timing enabled: its Lanczos kernels alone
                                (part of ms_small_la) */
} cdmd_info;

/* Validate `cfg`, prepare C (the sparse table is copied and reordered on the device)
   and allocate the device workspace on the current device.
   Errors: INVALID_ARG (constraints above, NULL table for SPARSE/SPIXEL, index out of
   range, sign not +/-1, k > min(p, m-1), unknown enum), UNSUPPORTED (precision
   combination not built), DEVICE (no gfx950 device), OUT_OF_MEMORY. */
cdmd_status cdmd_create(const cdmd_config* cfg, cdmd_model** out);

/* Algorithm 1 through the amplitudes on the video d_video (device, layout above, dtype of the
   configuration).  Synchronises `stream`.  Errors: INVALID_ARG (NULL),
   RANK_DEFICIENT, NUMERIC, DEVICE. */
cdmd_status cdmd_fit(cdmd_model* mdl, const void* d_video, void* stream);

/* Remark 3 (Section 3.2): amplitudes and selection on the compressed modes instead of the
   full modes.  space = CDMD_AMP_COMPRESSED: the next cdmd_fit computes no lift (the video
   is read twice per fit: the sketch, then the background / mask); b = argmin ||y_1 -
   Phi_Y b|| with Phi_Y = Y' V S^-1 W formed from the Gram of the sketch on the device,
   the canonical order uses |b_j| ||phi_Y,j||, cdmd_modes' phi_norm returns ||phi_Y,j||,
   and cdmd_select works on (Phi_Y, y_1) (x1_norm2 and omp_residual2 of cdmd_info then
   refer to y_1).  The background and mask still use the full modes X' G_S.  d_phi of
   cdmd_modes still gives the full modes.  CDMD_AMP_FULL (the default) restores eq. (eq:b) on the full modes.
   Takes effect at the next cdmd_fit (the model is marked unfitted).  Batches accept only
   models on the full modes.
   Errors: INVALID_ARG (NULL, unknown space), UNSUPPORTED (the model cannot use the device
   small linear algebra; a fit of a video that cannot, e.g. float32 or unaligned frames,
   also returns UNSUPPORTED), OUT_OF_MEMORY. */
cdmd_status cdmd_set_amplitudes(cdmd_model* mdl, int32_t space);

/* Dense Gaussian C (Section 3.3) kept in device memory.  on != 0: the library draws the
   p x n entries of the configured BF16 or FP8 form once (the same values, bit for bit,
   that the sketch otherwise draws on the fly) into memory it allocates and owns, and every
   later cdmd_fit streams them from HBM instead of drawing them.
   * BF16: bfloat16 bits stored pixel-major; each fit converts the video to exact bfloat16
     in S <= 32 pixel slices and forms the sketch as S batched library GEMMs (hipBLASLt,
     float32 accumulation and output) summed over the slices in float64.  Needs 2 p n + 2 m n
     bytes (plus padding to S slices of a multiple of 64 pixels) and S m p floats; the
     sketch equals the drawn form's up to the float32 summation order (not bit for bit).
   * FP8: e4m3 codes stored pixel-major; each fit splits every video byte u = 16 hi + lo
     into the two exact e4m3 codes of 16 hi and lo and forms the sketch as two batched
     library GEMMs (e4m3 inputs, float32 output, the second added into the first).  Needs
     p n + 2 m n bytes and S m p floats; equal to the drawn form's up to the summation order.
     Where the library offers no FP8 GEMM for the shape, the codes are stored row-major
     (rows padded to 64 pixels) and the sketch kernel reads them in place of its draws, bit
     for bit the drawn form.
   Models whose stored C goes through the library GEMM are refused by batches.
   on = 0 frees the copy.  Work goes on `stream`, which the call synchronises.  Errors:
   INVALID_ARG (NULL), UNSUPPORTED (not a Gaussian sketch in the BF16 or FP8 form, or no
   library GEMM for the shape), OUT_OF_MEMORY, DEVICE. */
cdmd_status cdmd_store_measurement(cdmd_model* mdl, int32_t on, void* stream);

/* Automatic target rank (Section 3.2, Remark 2): the optimal hard threshold of Gavish and
   Donoho (2014) for an unknown noise level, applied to the singular values of Y, the sketch
   of the snapshots X (eq. (eq:YCX)), in place of a given k.  d_video is sketched with cfg's
   measurement matrix (cfg->k is ignored), the float64 Gram of the sketch is formed on the
   device and its spectrum on the host (Householder tridiagonalisation, bisection);
   sigma_1 >= ... >= sigma_r are the r = min(p, m-1) singular values of Y, beta = r / max(p,
   m-1), tau* = omega(beta) median(sigma) with omega(beta) = lambda*(beta) / sqrt(mu_beta),
   lambda*(beta) = sqrt(2 (beta + 1) + 8 beta / ((beta + 1) + sqrt(beta^2 + 14 beta + 1)))
   and mu_beta the median of the Marchenko-Pastur law of ratio beta (numerical quadrature).
   *k_out = #{i : sigma_i > tau*} (0 when none; the caller clamps it to the k a model is
   created with, 1..40).  tau_out, sigma_out (r doubles, descending): optional.  Synchronises
   `stream`.  Errors: as cdmd_create and cdmd_fit, NUMERIC for a non-finite Gram. */
cdmd_status cdmd_optimal_rank(const cdmd_config* cfg, const void* d_video, void* stream, int32_t* k_out,
                              double* tau_out, double* sigma_out);

/* Results of the last fit, modes in canonical order (descending |b_j| ||phi_j||,
   conjugate partners with Im lambda > 0 first).  Each output is optional (NULL):
   lambda[2k] (re, im interleaved), b[2k] (re, im), sigma[k] (singular values of the
   scaled sketch Y, descending), phi_norm[k] (||phi_j||), and d_phi: device buffer of
   n*k complex64 (re, im float pairs), mode-contiguous: element (i, j) at j*n + i.
   Writing d_phi re-runs the lift on d_video (which must be the fitted video) and
   synchronises `stream`.  Errors: STATE (not fitted), INVALID_ARG. */
cdmd_status cdmd_modes(const cdmd_model* mdl, double* lambda, double* b, double* sigma,
                       double* phi_norm, const void* d_video, void* d_phi, void* stream);

/* Select background modes S and their amplitudes beta.
   selector OMP: K atoms (K >= 1, clamped to k).  OMEGA: threshold omega_thr > 0.
   EXPLICIT: explicit_idx[n_explicit] distinct canonical indices in [0, k).
   Outputs (optional): out_idx[k] receives S in selection order, out_n |S|,
   out_beta[2k] the complex amplitudes (re, im) in the order of out_idx.
   Errors: STATE (not fitted), INVALID_ARG, NUMERIC. */
cdmd_status cdmd_select(cdmd_model* mdl, int32_t selector, int32_t K, double omega_thr,
                        const int32_t* explicit_idx, int32_t n_explicit,
                        int32_t* out_idx, int32_t* out_n, double* out_beta);

/* Write the background of frames [t0, t1) (0-based, t1 <= m) to d_L (device float32,
   frame-major, frame t0+s at s*ldL, ldL >= n), or, if static_bg, the static model
   xhat (n floats) to d_L.  Needs the fitted video again (the modes are recomputed
   from X' on the fly).  Errors: STATE (not selected), INVALID_ARG, NUMERIC. */
cdmd_status cdmd_background(const cdmd_model* mdl, const void* d_video, int64_t t0,
                            int64_t t1, int32_t static_bg, float* d_L, int64_t ldL,
                            void* stream);

/* Foreground mask of all m frames: mask_jt = |x_jt - L_jt| > tau (strict; NaN -> 0),
   L the dynamic background of the selected modes, or the static model if static_bg.
   bitpacked = 1: d_mask holds uint32 words, frame t at t*ceil(n/32), pixel i of the
   frame in bit (i mod 32) of word i/32 (unused high bits zero).  bitpacked = 0: one
   uint8 (0/1) per pixel, frame t at t*n.  h_counts (optional, host int64[m]) receives
   the foreground pixel count per frame.  Enqueued on `stream`; synchronises only if
   h_counts is given.  Errors: STATE (not selected), INVALID_ARG, NUMERIC. */
cdmd_status cdmd_foreground(const cdmd_model* mdl, const void* d_video, float tau,
                            int32_t static_bg, int32_t bitpacked, void* d_mask,
                            int64_t* h_counts, void* stream);

/* Post-processing of foreground masks (Section 4, the evaluation on the BMC videos: the
   thresholded mask, then median filtered): 3x3 median of each of the m frames' binary
   H x W masks (pixel i = y W + x), i.e. the majority of the nine neighbours, with rows and
   columns beyond the border replicated from the edge.  Layout as cdmd_foreground writes
   it: bitpacked = 1 uint32 words, frame t at t*ceil(HW/32); bitpacked = 0 one uint8 (0/1)
   per pixel, frame t at t*HW.  d_in and d_out are device buffers that must not overlap.
   Enqueued on `stream`.  Errors: INVALID_ARG (NULL, sizes, m > 65535, overlap),
   UNSUPPORTED (H W >= 2^31), DEVICE. */
cdmd_status cdmd_mask_median3(const void* d_in, void* d_out, int64_t H, int64_t W, int64_t m,
                              int32_t bitpacked, void* stream);

/* ---- tile shapes and batches ---------------------------------------------------------
   cdmd_autotune times candidate tile shapes of the model's size class on d_video (the
   number of persistent lift workgroups; for the dense Gaussian sketch the number of
   pixel slices; for the sparse sketch of an aligned uint8 video the gather or streaming
   form and its shape), keeps the fastest for the model and caches the choice per size
   class for the process.  Synchronises `stream`.  Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
cdmd_status cdmd_autotune(cdmd_model* mdl, const void* d_video, void* stream);

/* A batch fits many models (streams of different resolution, frame count, rank and
   sketch) with one graph launch: the sketch and Gram of every model and then its lift run
   on a pool of streams, and the small linear algebra of all models is one launch with a
   workgroup per model (Algorithm 1 for each stream; the paper processes independent
   200-frame batches the same way, Section 4).  The graph is captured on the first
   cdmd_batch_fit (after cdmd_autotune of every model not yet tuned) and replayed while
   the video pointers and the stream stay the same.  Models whose fit needs the host small
   linear algebra (float32 videos, unaligned frames, m > 1025) are fitted one after the
   other after the graph.  The batch borrows the models (free them after the batch). */
typedef struct cdmd_batch cdmd_batch;
/* Errors: INVALID_ARG (NULL or repeated model, n < 1), OUT_OF_MEMORY, DEVICE. */
cdmd_status cdmd_batch_create(cdmd_model* const* models, int32_t n, cdmd_batch** out);
/* d_videos[i] is the video of models[i].  per_model (optional, n entries) receives each
   model's status (STATE for a model not attempted because the batch failed first); the
   call returns OK when all succeed, else the first failure.  The graph runs on a stream
   of the batch's own, after the work already enqueued on `stream`.
   Synchronises `stream`.  Errors: INVALID_ARG, DEVICE, and the per-model errors of
   cdmd_fit. */
cdmd_status cdmd_batch_fit(cdmd_batch* batch, const void* const* d_videos, void* stream,
                           cdmd_status* per_model);
/* The foreground masks of every model of the batch (Section 4, eq. (eq:thres), on the
   reconstruction of eq. (equ:DMDTerms) with the selected modes), as cdmd_foreground with
   bitpacked = 1 for each, in one work-queue launch over the (model, pixel tile) pairs of
   all models of a reconstruction form and tile size (at most 64 models each) instead of
   one launch per model: the Vandermonde
   operands of each model are formed on the device, then every tile of every model is
   reconstructed and thresholded.  d_videos[i] is the video models[i] was fitted on,
   d_masks[i] its mask (device, ceil(n_i/32) uint32 words per frame, m_i frames, the
   layout of cdmd_foreground).  Each mask equals cdmd_foreground's bit for bit.  Models
   whose reconstruction takes the VALU form (more than 16 selected modes, float32 videos,
   too many frames for the tile in LDS) are launched one by one.  Every model must have
   been selected (cdmd_select or cdmd_select_learned).  Enqueued on `stream`; does not
   synchronise it (a later call waits on the device for this one's work lists, and on the
   host only for their copy).  Errors: INVALID_ARG (NULL argument, tau < 0), STATE (a
   model not selected), NUMERIC (|lambda|^(m-1) overflow), DEVICE. */
cdmd_status cdmd_batch_foreground(cdmd_batch* batch, const void* const* d_videos, float tau,
                                  int32_t static_bg, void* const* d_masks, void* stream);
void cdmd_batch_free(cdmd_batch* batch);

/* ---- long videos -------------------------------------------------------------------
   Section 4 splits a long video into batches of consecutive frames and decomposes each on
   its own (the paper uses 200 frames, a very sparse C with p = 1000, the automatic rank of
   Remark 2 and OMP with K = 10).  cdmd_process_video does that for `frames` frames at
   d_video (layout and dtype of `base`, frame stride base->ld; base->m and base->k are
   ignored): every batch is fitted with the configuration `base` (the same C), its
   background selected by OMP with K atoms, and its foreground mask (bit-packed, the
   layout of cdmd_foreground) written to the rows of d_mask (frames x ceil(n/32) words)
   of its frames; with H, W set, each mask is 3x3-median filtered (cdmd_mask_median3).
   Batches hold batch_frames frames, the last the remainder (a single trailing frame
   joins the batch before it).  `workers` host threads, each with its own stream and
   models, take the batches in turn, so up to `workers` batches are in flight and the
   small linear algebra of one overlaps the streaming kernels of another.  k = 0 chooses
   the rank of every batch by Remark 2, clamped to [1, min(m_b - 1, p, 40)] (k_used, host, one
   entry per batch, at most ceil(frames / batch_frames), receives the ranks when not NULL).
   The call waits for `stream` (the video's producer) and returns when every mask is
   written.  Errors: INVALID_ARG, the errors of cdmd_create / cdmd_fit / cdmd_select /
   cdmd_foreground for the first batch that failed (its message names it). */
typedef struct {
  int32_t batch_frames;  /* frames per batch, >= 2 */
  int32_t k;             /* target rank of every batch, or 0: per batch by Remark 2 */
  int32_t K;             /* OMP atoms of the background selection */
  int32_t workers;       /* batches in flight, 1..4 */
  double tau;            /* foreground threshold (eq. (eq:thres)) */
  int64_t H, W;          /* frame shape for the median filter (H * W = n), or 0, 0 */
} cdmd_video_plan;

cdmd_status cdmd_process_video(const cdmd_config* base, const cdmd_video_plan* plan, const void* d_video,
                               int64_t frames, void* d_mask, int32_t* k_used, void* stream);

/* The same as a reusable executor: cdmd_process_video is cdmd_video_create, one
   cdmd_video_run and cdmd_video_free.  The executor owns its worker streams, the models
   of every (batch length, rank) it has met and the unfiltered-mask buffers, and keeps
   them from one run to the next, so later videos of the same shape allocate nothing.
   cdmd_video_create copies `base` and its sparse table (the caller's arrays may be freed
   afterwards) and checks the plan (INVALID_ARG); models are created on first use, so
   configuration errors of `base` surface in the first cdmd_video_run.  cdmd_video_run
   takes `frames` frames at d_video with the layout of `base` and behaves as
   cdmd_process_video; it works on the device that was current at cdmd_video_create and
   leaves the caller's current device as it found it; runs on one executor must not
   overlap (one host thread at a time).  cdmd_video_free waits for the executor's streams
   and releases everything (NULL is a no-op). */
typedef struct cdmd_video cdmd_video;
cdmd_status cdmd_video_create(const cdmd_config* base, const cdmd_video_plan* plan, cdmd_video** out);
cdmd_status cdmd_video_run(cdmd_video* video, const void* d_video, int64_t frames, void* d_mask, int32_t* k_used,
                           void* stream);
void cdmd_video_free(cdmd_video* video);

/* ---- learned background selector -------------------------------------------------
   A 6-64-64-1 network with GELU activations (exact erf) maps per-mode features to the
   logit of "sparse coding selects this mode"; the paper suggests learning the background
   amplitude profile instead of a fixed rule (Section 2.2, "DMD for Foreground/Background
   Separation", its last paragraph).  Parameters: one flat float32 vector of CDMD_MLP_NPARAM numbers, W1 (64 x 6
   row-major), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3.  Features of mode j (canonical
   order, k modes, m frames): |lambda_j|, |arg lambda_j|, log(|b_j| ||phi_j|| / ||x_1||),
   ||phi_j|| / max_i ||phi_i||, (1/m) sum_t |b_j|^2 |lambda_j|^{2t} ||phi_j||^2 / ||x_1||^2,
   j / k.  The amplitude and mode norm enter relative to the first frame and to the
   largest mode, so that the features do not depend on the frame size or the scale of C.
   All pointers named d_* are device memory owned by the caller; work goes on `stream`
   (NULL = default stream) and the calls return after enqueueing unless stated. */
#define CDMD_MLP_NPARAM 4673

/* Features of the k modes of the last fit into d_feats (float32, k x 6 row-major).
   Errors: STATE (not fitted), INVALID_ARG, DEVICE. */
cdmd_status cdmd_mode_features(const cdmd_model* mdl, float* d_feats, void* stream);

/* Mean binary cross-entropy with logits over n samples (d_X: n x 6, d_y: n labels in
   {0, 1}) and its gradient with respect to the parameters: d_grad[CDMD_MLP_NPARAM],
   d_loss[1] (either may be NULL).  Deterministic (fixed-order sums).  Synchronises
   `stream`.  Errors: INVALID_ARG (n < 1, NULL inputs), OUT_OF_MEMORY, DEVICE. */
cdmd_status cdmd_mlp_grad(const float* d_params, const float* d_X, const float* d_y, int32_t n,
                          float* d_grad, float* d_loss, void* stream);

/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on batches of
   `batch` samples: step s uses the rows d_batch_idx[s*batch .. s*batch + batch - 1] of
   d_X / d_y (n_samples rows; device int32 indices, caller-drawn; an index outside
   [0, n_samples) contributes nothing).  d_adam_m, d_adam_v: the moment vectors
   (CDMD_MLP_NPARAM each, zero before the first step); step0: Adam steps already taken
   (bias correction).  d_losses (optional): the mean batch loss of every step.
   Synchronises `stream`.  Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
cdmd_status cdmd_mlp_train(float* d_params, float* d_adam_m, float* d_adam_v, const float* d_X,
                           const float* d_y, int64_t n_samples, const int32_t* d_batch_idx,
                           int32_t batch, int32_t steps, float lr, int64_t step0, float* d_losses,
                           void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): cdmd_mlp_train with the same arguments
   and results, except that the per-batch partial gradients live in a static scratch
   array the library holds on each device until the process ends, so the call allocates
   nothing and does not synchronise (it returns after enqueueing on `stream`).  batch is at
   most CDMD_MLP_NOALLOC_MAX_BATCH.  Every call on one device shares that device's
   scratch: calls that overlap on one device (other streams or threads) race.
   Errors: INVALID_ARG (including batch above the maximum), DEVICE. */
#define CDMD_MLP_NOALLOC_MAX_BATCH 1024
cdmd_status cdmd_mlp_train_noalloc(float* d_params, float* d_adam_m, float* d_adam_v, const float* d_X,
                                   const float* d_y, int64_t n_samples, const int32_t* d_batch_idx,
                                   int32_t batch, int32_t steps, float lr, int64_t step0, float* d_losses,
                                   void* stream);

/* Logits of n samples (d_X: n x 6) into d_logits; bf16 != 0 rounds the hidden activations
   and the weights after the input layer to bfloat16 (float32 accumulation; the input layer,
   which carries the features' standardisation, stays float32).  Errors: INVALID_ARG,
   DEVICE. */
cdmd_status cdmd_mlp_forward(const float* d_params, const float* d_X, int32_t n, int32_t bf16,
                             float* d_logits, void* stream);

/* Learned selection for the last fit: the network (bfloat16 inference) gives each mode a
   probability p_j; when every mode is confident, max(p_j, 1 - p_j) >= confidence, the
   support is {j : p_j >= 1/2} with beta refitted by least squares (as EXPLICIT);
   otherwise, or when that support is empty, orthogonal matching pursuit with K_fallback
   atoms decides (*used_fallback = 1).  Outputs as cdmd_select; prob (optional, host
   float64[k]) receives p.  Synchronises `stream`.  Errors: STATE, INVALID_ARG, NUMERIC,
   DEVICE. */
cdmd_status cdmd_select_learned(cdmd_model* mdl, const float* d_params, double confidence,
                                int32_t K_fallback, int32_t* out_idx, int32_t* out_n,
                                double* out_beta, double* prob, int32_t* used_fallback,
                                void* stream);

/* Sketch of the last fit, Y^ = C D (p x m), scaled (u/255 for uint8, 1/sqrt(p) for
   Gaussian and SRFT), host float64, frame-major: element (r, t) at t*p + r; for the
   complex SRFT sketch 2 p m numbers, the real and imaginary part of (r, t) at
   t*2p + 2r and t*2p + 2r + 1.  Optional
   h_int (host int64[p*m]): the exact integer sums of a sparse/single-pixel sketch of
   a uint8 video before scaling (INVALID_ARG otherwise).  Errors: STATE. */
cdmd_status cdmd_get_sketch(const cdmd_model* mdl, double* h_Y, int64_t* h_int);

/* Counters and timings of the last calls (see cdmd_info).  Reading gpu_ms_recon waits
   for the last reconstruction launch to finish. */
cdmd_status cdmd_info_get(const cdmd_model* mdl, cdmd_info* info);

/* Enable (1) or disable (0) HIP-event timing of the kernel groups of this model. */
cdmd_status cdmd_set_timing(cdmd_model* mdl, int32_t enable);

/* Release the model and its device memory.  NULL is a no-op. */
void cdmd_free(cdmd_model* mdl);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* cdmd_last_error(void);

int32_t cdmd_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CDMD_H */
