/*
 * lfrl.h - C ABI of the MI355X (gfx950) light-field Richardson-Lucy library.
 *
 * The library deconvolves a light-field microscopy image into a volume of
 * axial layers with Richardson-Lucy iterations run entirely on the GPU, and
 * scores each iterate with the DCT-entropy image-quality metric that picks the
 * stopping iteration (AutoDeconJ, arXiv 2208.11422: sec. 1 and sec. 2.1 for
 * the GPU-resident deconvolution, sec. 2.2 / Eqs. 1-12 for the metric).
 *
 * Conventions for every call:
 *   - Pointers are DEVICE pointers on the plan's device unless marked [host].
 *   - Arrays are row-major, contiguous float32 (metric results float64):
 *       PSF    psf[nz][nnum][nnum][K][K]: image of a point source in depth plane
 *              j whose pixel has row phase a = r mod nnum and column phase
 *              b = s mod nnum; tap (u, v) lies at displacement (u - c0, v - c0)
 *              from the source pixel, c0 = (K - 1) / 2, K odd.
 *       volume vol[nz][h][w]; image img[h][w]; h and w multiples of nnum, the
 *              lenslet grid starting at pixel (0, 0).
 *   - Projections are linear with zero padding outside the image ("same" size,
 *     not circular).
 *   - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *     NULL = the null stream) unless stated otherwise.
 *   - The caller owns every buffer it passes.  A plan owns its PSF spectra and
 *     its workspace; after lfrl_plan returns, no call allocates device memory
 *     except lfrl_metric / lfrl_metric_ex (see there) and the job calls (a
 *     job's state is allocated by lfrl_job_create, sized by
 *     lfrl_job_footprint).
 *   - One call at a time per plan (calls on one plan share its workspace).
 *   - Calls return LFRL_OK or a negative lfrl_status and never throw.  Argument
 *     errors are reported before anything is launched; lfrl_last_error() gives
 *     a message (per thread).  Outputs are undefined after an error.
 */
#ifndef LFRL_H
#define LFRL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lfrl_plan_s *lfrl_plan_t;

typedef enum {
    LFRL_OK = 0,
    LFRL_ERR_ARG = -1,          /* bad argument or size */
    LFRL_ERR_NOMEM = -2,        /* device allocation failed */
    LFRL_ERR_DEVICE = -3,       /* HIP runtime / kernel launch error */
    LFRL_ERR_UNSUPPORTED = -4,  /* valid request the library does not serve */
    LFRL_ERR_NUMERIC = -5       /* non-finite value met where one is not allowed */
} lfrl_status;

typedef enum {
    LFRL_FP32 = 0,        /* spectra, tile DFTs and contractions in float32 */
    LFRL_SPLIT_FP16 = 1,  /* PSF spectra stored in FP16 (per-frequency power-of-two
                             scale; half the bytes streamed per projection); tile
                             spectra split into hi + lo FP16 parts, products on
                             FP16 matrix cores with FP32 accumulation; tile DFTs,
                             ratio and update in float32.  Relative error of a
                             projection about 1e-5 to 1e-4 instead of 1e-7. */
    LFRL_SPLIT_BF16 = 2   /* as LFRL_SPLIT_FP16 with BF16 storage and BF16 matrix
                             cores: 8 significant bits per spectrum value (FP16:
                             11), so errors about 8 times larger.  The RL iterates
                             drift from the float64 result by about 1e-5 more per
                             iteration: measured within 1e-3 relative up to about
                             35 iterations, 1.2e-3 at 50 (FP16 stays near 1e-4);
                             choose FP16 or FP32 for longer runs at that bar. */
} lfrl_precision;

/* Plan flags.  LFRL_PLAN_AUTOTUNE (with tile_q = 0): time the best few tile
 * sides by the model on the device (one forward and one back projection of
 * max_batch largest frames each, on zero spectra) and keep the fastest.
 * LFRL_NORMALIZE_PSF: scale every (j, a, b) kernel of the plan's copy of the
 * PSF set to unit sum (sums in float64, one rounding to float32) before
 * anything is built from it; a kernel whose sum is not positive is kept as it
 * is.  The caller's psf array is not modified. */
enum { LFRL_PLAN_AUTOTUNE = 1u << 0, LFRL_NORMALIZE_PSF = 1u << 1 };

/* Plan description.  Geometry of the PSF set and the largest image the plan
 * serves (the memory estimate of Fig. 1 is made for that size). */
typedef struct {
    int32_t nnum;      /* pixels per lenslet per axis, N >= 1 */
    int32_t nz;        /* depth planes, >= 1 */
    int32_t ksize;     /* PSF support per axis, odd, >= 1 */
    int32_t max_h;     /* largest image height served, multiple of nnum */
    int32_t max_w;     /* largest image width served, multiple of nnum */
    int32_t precision; /* lfrl_precision */
    int32_t tile_q;    /* DFT tile side in lenslets; 0 = choose from the model */
    uint32_t flags;    /* LFRL_PLAN_AUTOTUNE | LFRL_NORMALIZE_PSF, or 0 */
    int32_t max_batch; /* frames of max_h x max_w whose tiles one batched
                          projection covers (lfrl_job_step); 0 or 1 = one
                          frame, at most 16.  Workspace grows with it. */
} lfrl_plan_desc;

/* Read-only facts about a plan (all [host]). */
typedef struct {
    int32_t tile_q;        /* DFT tile side Q (lenslets) */
    int32_t tile_out;      /* output lenslets per tile side T = Q - R + 1 */
    int32_t taps;          /* polyphase taps per side R */
    int32_t nfreq;         /* half-spectrum frequencies per tile, Q * (Q/2 + 1) */
    int32_t max_tiles;     /* tiles one projection covers: max_batch frames of
                              the plan's largest image */
    int32_t split_k;       /* reduction split of the forward contraction */
    size_t resident_bytes; /* spectra held for the plan's lifetime */
    size_t workspace_bytes;/* workspace: tile spectra for max_tiles tiles plus
                              the frame state of lfrl_deconvolve */
    int32_t tune_candidates; /* tile sides timed (autotuned plans), else 0 */
    double tune_ms;        /* measured forward + back projection of max_batch
                              largest frames at the chosen side, else 0 */
    int32_t nfreq_unique;  /* frequencies the contractions visit: nfreq less the
                              conjugates of others on the kv = 0 and kv = Q/2
                              columns of the Hermitian half spectrum */
} lfrl_plan_info_t;

/* Memory estimate before allocation (Fig. 1: the required memory is
 * estimated before anything is placed on the card).  [host], no device work.
 * Either output pointer may be NULL.  With LFRL_PLAN_AUTOTUNE the figures are
 * the largest over the tile sides the tuner may choose. */
int lfrl_plan_footprint(const lfrl_plan_desc *desc, size_t *resident_bytes,
                        size_t *workspace_bytes);

/* Build a plan: validate `desc`, allocate spectra and workspace, and turn the
 * PSF set into the resident per-frequency spectra the projections stream
 * (Fig. 1: the PSF is placed on the card once and used directly by every
 * later reconstruction).  `psf` is [nz][nnum][nnum][K][K] float32; the caller
 * may free it once the work queued on `stream` has completed.  On success
 * *out receives the plan; on error *out is set to NULL. */
int lfrl_plan(lfrl_plan_t *out, const lfrl_plan_desc *desc, const float *psf,
              void *stream);

/* Release a plan and everything it owns (synchronises its device first).
 * NULL is accepted. */
int lfrl_plan_destroy(lfrl_plan_t plan);

/* Fill *info with the plan's tile shape and memory figures. */
int lfrl_plan_get_info(lfrl_plan_t plan, lfrl_plan_info_t *info);

/* Forward light-field projection img = A vol (sec. 1; the model behind RL):
 * img[p] = sum_j sum_q vol[j][q] * psf[j][q mod N][p - q + c0]  (2-D indices),
 * i.e. every depth and every lenslet-relative phase convolved with its own PSF
 * and summed into one image.  vol [nz][h][w] -> img [h][w]; h <= max_h,
 * w <= max_w, both multiples of nnum. */
int lfrl_forward(lfrl_plan_t plan, int32_t h, int32_t w, const float *vol,
                 float *img, void *stream);

/* Back projection with the transposed PSFs, vol = A^T img, the exact adjoint
 * of lfrl_forward: vol[j][q] = sum_p img[p] * psf[j][q mod N][p - q + c0].
 * img [h][w] -> vol [nz][h][w]. */
int lfrl_backward(lfrl_plan_t plan, int32_t h, int32_t w, const float *img,
                  float *vol, void *stream);

/* Stop modes of lfrl_deconvolve. */
typedef enum {
    LFRL_STOP_NONE = 0,   /* run max_iters iterations, no metric */
    LFRL_STOP_METRIC = 1, /* metric every iteration; stop when it decreases */
    LFRL_STOP_TRACK = 2   /* metric every iteration and keep the best iterate,
                             but always run max_iters iterations */
} lfrl_stop_mode;

/* Update rules of lfrl_deconvolve. */
typedef enum {
    LFRL_UPDATE_RL = 0,  /* Richardson-Lucy: x * A^T(y / (A x + b)) / A^T 1 */
    LFRL_UPDATE_ISRA = 1 /* ISRA: x * A^T y / A^T(A x + b) (least squares) */
} lfrl_update;

/* Coefficient regions of the DCT entropy. */
typedef enum {
    LFRL_REGION_TRIANGLE = 0,  /* u / xs + v / ys < 1 (Eq. 6), prefactor 2 / (xs ys) */
    LFRL_REGION_RECTANGLE = 1, /* u < xs and v < ys (Eq. 12's limits), 1 / (xs ys) */
    LFRL_REGION_WHOLE = 2      /* every coefficient (Fig. 2(c)'s overall value),
                                  1 / (w h); xs and ys are ignored */
} lfrl_region;

/* The 2-norm the coefficients are divided by. */
typedef enum {
    LFRL_NORM_MATRIX = 0,  /* Frobenius norm of the whole coefficient matrix */
    LFRL_NORM_REGION = 1,  /* Frobenius norm of the coefficients in the region */
    LFRL_NORM_SPECTRAL = 2 /* largest singular value of the coefficient matrix
                              (equal to the image's: the DCT is orthonormal),
                              by float64 Lanczos iteration; h + w <= 6144.
                              Images of 16384 pixels and more spread it over
                              up to 32 workgroups that exchange partial sums
                              through device memory and must be resident
                              together; should they not be (a device crowded
                              by other kernels), a bounded wait gives up and
                              the metric is NaN instead of a hang */
} lfrl_norm;

typedef struct {
    int32_t max_iters; /* iteration cap, >= 1 */
    int32_t stop;      /* lfrl_stop_mode */
    int32_t patience;  /* consecutive strict decreases that stop (>= 1) */
    int32_t init;      /* 0 = start from ones, 1 = start from the caller's vol,
                          2 = start from the back projection A^T img */
    double xs, ys;     /* legs of the triangular DCT region, in DCT bins:
                          X_S along the width, Y_S along the height (Eq. 6) */
    /* Variants (a zero-filled tail gives the method as the paper states it). */
    int32_t update;    /* lfrl_update */
    int32_t region;    /* lfrl_region of the metric */
    int32_t norm;      /* lfrl_norm of the metric */
    int32_t window;    /* the stop rule compares means of the last `window`
                          metric values (0 or 1: the values themselves) */
    double background; /* known constant background b >= 0 of the image model
                          A x + b */
} lfrl_rl_opts;

typedef struct {
    int32_t iters_run; /* iterations executed */
    int32_t best_iter; /* iteration whose volume was returned */
    int32_t stopped;   /* 1 if the stop rule fired before the cap */
    int32_t weak_voxels; /* voxels updated by exact float64 window sums (their
                            A^T 1 is below 1e-2 of the largest, so the tile-DFT
                            values would be dominated by round-off) */
    double *metric_trace; /* [host] array of max_iters or NULL: e_1, e_2, ... */
    double *flux_trace;   /* [host] array of max_iters or NULL:
                             <A^T 1, x^k> / sum(img) - 1 for each iterate */
} lfrl_rl_report;

/* Richardson-Lucy deconvolution (sec. 1; all iterations on the GPU and only
 * the result handed back, sec. 2.1):
 *   x^0 = 1 (or vol, or A^T img), c = A^T 1,
 *   x^k = x^{k-1} * A^T( img / (A x^{k-1} + b) ) / c,
 * with img / (A x + b) := 0 where A x + b <= 0 and x := 0 where c <= 0
 * (b = opts->background, 0 by default).  With opts->update = ISRA instead
 *   x^k = x^{k-1} * A^T img / A^T(A x^{k-1} + b),  := 0 where A^T(A x + b) <= 0.
 * With a metric stop mode, every iterate is scored by the DCT entropy of its
 * z maximum projection (lfrl_metric_ex with opts->region and opts->norm) and
 * the stop rule of sec. 2.2 applies: stop once the entropy (or the mean of its
 * last opts->window values) has strictly decreased `patience` times in a row
 * and return the iterate with the largest entropy seen (ties: the later one).
 * img [h][w] -> vol [nz][h][w] (x^{best_iter}, or x^{max_iters} without a
 * metric).  With LFRL_STOP_METRIC the iterations are queued in chunks of 4
 * ahead of the host's reading of the stop rule (each chunk replayed from a
 * captured graph); the kernels of iterations after the stop return at once,
 * so the result is that of a run that reads the rule after every iteration.
 * Synchronises `stream` before returning (the host needs the stop decision
 * and the report).  `report` [host] may be NULL.  The weakly
 * observed voxels are listed when A^T 1 is first formed for an image size; if
 * more than min(nz h w, 2^20) of them remain below even 1e-9 of the largest
 * A^T 1 (a depth plane with an all-zero PSF, say), the call returns
 * LFRL_ERR_UNSUPPORTED rather than leave some of them on the inexact path. */
int lfrl_deconvolve(lfrl_plan_t plan, int32_t h, int32_t w, const float *img,
                    float *vol, const lfrl_rl_opts *opts, lfrl_rl_report *report,
                    void *stream);

/* ---- batched and served deconvolution --------------------------------------
 * A job is one frame's Richardson-Lucy run (the iteration and stop rule of
 * lfrl_deconvolve) held on the device between calls: its own copy of the
 * image, the iterates, A^T 1 with its weakly observed voxels, and the metric
 * and stop state.  lfrl_job_step advances many jobs by one iteration each.
 * Jobs on one plan share every launch of the projections: their tiles are
 * concatenated along the contraction's tile dimension, so the plan's spectra
 * stream from memory once per projection for the whole batch (up to
 * max_batch largest frames, or 16 frames, per launch).  Jobs on different
 * plans run side by side on internal streams.  A job's iterates do not depend
 * on which other jobs share its steps.  Calls on jobs of one plan, and that
 * plan's other calls, must not overlap (they share its workspace). */
typedef struct lfrl_job_s *lfrl_job_t;

enum { LFRL_JOB_FLUX = 1u << 0 }; /* record the flux trace of the report */

/* Device bytes lfrl_job_create allocates for an h x w frame on `plan` (the
 * admission figure of a serving loop, in the spirit of Fig. 1's estimate
 * before allocation).  [host], no device work. */
int lfrl_job_footprint(lfrl_plan_t plan, int32_t h, int32_t w, size_t *bytes);

/* Create a job for image img [h][w] (copied; the caller may reuse img once
 * the call returns) with the options of lfrl_deconvolve.  vol0 [nz][h][w] is
 * the start volume when opts->init == 1 (copied), else ignored.  Computes A^T 1
 * for the frame (and A^T img for the ISRA update or the back projection start)
 * and synchronises `stream`.  Returns LFRL_ERR_NUMERIC, and
 * creates nothing, when img holds a negative or non-finite value;
 * LFRL_ERR_NOMEM when the job's memory cannot be allocated;
 * LFRL_ERR_UNSUPPORTED when the frame has more weakly observed voxels than
 * their list holds (see lfrl_deconvolve). */
int lfrl_job_create(lfrl_job_t *out, lfrl_plan_t plan, int32_t h, int32_t w,
                    const float *img, const float *vol0, const lfrl_rl_opts *opts,
                    uint32_t flags, void *stream);

/* One Richardson-Lucy iteration for every listed job that is not done (a job
 * is done at its iteration cap, or, with LFRL_STOP_METRIC, once the stop rule
 * fired).  Synchronises `stream` when a listed job uses LFRL_STOP_METRIC (the
 * host needs the decision); otherwise only queues work.  *active (may be
 * NULL) receives the number of listed jobs not yet done. */
int lfrl_job_step(const lfrl_job_t *jobs, int32_t njobs, int32_t *active, void *stream);

/* Host-side state as of the last step: done flag and iterations run. */
int lfrl_job_poll(lfrl_job_t job, int32_t *done, int32_t *iters_run);

/* Copy the job's result (the iterate lfrl_deconvolve would return after the
 * same iterations) into vol [nz][h][w] (may be NULL) and fill `report` [host]
 * (may be NULL).  Synchronises `stream`. */
int lfrl_job_result(lfrl_job_t job, float *vol, lfrl_rl_report *report, void *stream);

/* Release a job (NULL accepted).  Call once no queued work uses it
 * (lfrl_job_result synchronises its stream), and before destroying its plan. */
int lfrl_job_destroy(lfrl_job_t job);

/* Deconvolve n frames, each on its own plan (plans may repeat) and size, as
 * jobs stepped together until all are done; vols[i] [nz_i][h_i][w_i] receives
 * frame i's result and reports[i] (array may be NULL) its report.  Allocates
 * the jobs' state for the duration of the call; synchronises `stream`. */
int lfrl_deconvolve_batch(const lfrl_plan_t *plans, int32_t n, const int32_t *h,
                          const int32_t *w, const float *const *imgs, float *const *vols,
                          const lfrl_rl_opts *opts, lfrl_rl_report *reports, void *stream);

/* DCT entropy of a 2-D image (sec. 2.2, Eqs. 1-6 and 12): F = orthonormal
 * DCT-II of img (Eqs. 1-4), n = Frobenius norm of F (the "2-norm of a matrix"),
 * S = {(u, v): u / xs + v / ys < 1} with u the width and v the height
 * frequency, and
 *     *out = -(2 / (xs * ys)) * sum_{(u,v) in S} |F/n| log2 |F/n|
 * with 0 log 0 = 0 (0 for an all-zero image).  Pass nz > 1 to score the z
 * maximum projection of a volume img[nz][h][w] instead.  `out` is a device
 * float64.  Uses a per-device scratch buffer that the library allocates on
 * first use and grows when a larger image needs it.  Calls on one device share
 * that buffer: each call's kernels wait (on its stream) for the previous
 * call's, so calls on different streams are serialised on the device. */
int lfrl_metric(int32_t nz, int32_t h, int32_t w, const float *img, double xs,
                double ys, double *out, void *stream);

/* lfrl_metric with a choice of region (lfrl_region) and norm (lfrl_norm):
 *     *out = -(1 / G) * sum_{(u,v) in S} |F/n| log2 |F/n|,
 * G the area of S (xs ys / 2, xs ys, or w h) and n the Frobenius norm of F
 * over the whole matrix or over S, or its spectral norm.  The triangle and the rectangle need legs
 * of at most 256 bins; the whole region takes any image. */
int lfrl_metric_ex(int32_t nz, int32_t h, int32_t w, const float *img, double xs, double ys,
                   int32_t region, int32_t norm, double *out, void *stream);

/* lfrl_metric_ex without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, kernels and results (bit for bit) as
 * lfrl_metric_ex, but the scratch is a fixed array in the library's device
 * memory (about 25 MiB per GPU the library runs on, held until the process
 * ends) instead of a growable buffer.  Limits: h <= 1024 and w <= 1024, region
 * LFRL_REGION_TRIANGLE or LFRL_REGION_RECTANGLE (legs of at most 256 bins);
 * anything larger or LFRL_REGION_WHOLE returns LFRL_ERR_UNSUPPORTED before any
 * launch.  Every call on one GPU uses that GPU's one array, and its contents
 * persist between calls (each call rebuilds everything it reads): calls that
 * overlap on one GPU (on different streams, or from different host threads
 * without an ordering between them) race on it and may return wrong values, so
 * the caller must serialise them.  Calls on one stream are ordered and safe. */
int lfrl_metric_noalloc(int32_t nz, int32_t h, int32_t w, const float *img, double xs,
                        double ys, int32_t region, int32_t norm, double *out, void *stream);

/* Triangle legs from the optics (Eqs. 7, 9-11), [host]:
 * P_u = d_ml / (mag * nnum), d_psf = 1.22 * lambda * nnum / na,
 * xs = P_u * w / d_psf, ys = P_u * h / d_psf.  Lengths in one unit. */
int lfrl_metric_cutoff(double d_ml, double mag, int32_t nnum, double lambda,
                       double na, int32_t h, int32_t w, double *xs, double *ys);

/* ---- PSF from optical parameters (sec. 2.1, Fig. 1) ----------------------
 * The PSF set of a light-field microscope computed on the GPU from its optics
 * (Fig. 1: computing it from the system's parameters is the default source;
 * sec. 2.1: the time-consuming parts of the PSF computation run on the GPU).
 * Scalar wave-optics model, all lengths in one unit:
 *   1. field on the native image plane (at the lenslet array) of a point
 *      source on the axis at depth z, from the Debye integral of an objective
 *      obeying the sine condition:
 *        U(r) = int_0^alpha sqrt(cos t) sin t exp(i k n z (1 - cos t))
 *                             J0(k n r sin t / mag) dt,
 *      alpha = asin(na / n_medium), k = 2 pi / wavelength, r the image-plane
 *      radius; Gauss-Legendre quadrature with nquad nodes (0: 1024);
 *      constant factors and the phase common to a depth are dropped;
 *   2. each lenslet's thin-lens phase exp(-i pi |x - c|^2 / (wavelength f_ml))
 *      about its centre c; lenslet l covers sensor pixels l*nnum ..
 *      l*nnum + nnum - 1 of each axis (the projections' phase convention);
 *   3. Fresnel propagation over f_ml with the transfer function
 *      exp(-i pi wavelength f_ml (fx^2 + fy^2));
 *   4. intensity |U|^2 summed over the osr x osr field samples of each pixel.
 * Sampling: pixel pitch d_ml / nnum, field samples osr per pixel per axis; a
 * window of ksize x ksize pixels (G = ksize * osr samples) centred on the
 * source pixel, zero-padded to the smallest 2^a 3^b 5^c >= G for the periodic
 * propagation (the window at offset (Gf - G) / 2).  The source of phase (a, b)
 * sits at the centre of pixel (a, b) of its lenslet, at depth depths[j].
 * Out: psf [nz][nnum][nnum][ksize][ksize] float32 (device), the layout
 * lfrl_plan takes; with LFRL_PSF_UNIT_SUM each (j, a, b) kernel is scaled to
 * unit sum (float64 sums).  Field DFTs run in float32, the quadrature sums in
 * float64.  Limits: ksize * osr <= 2048.  Allocates its scratch (the Debye
 * table and up to 1 GiB of field buffers) and frees it before returning;
 * synchronises `stream`.  Argument errors: LFRL_ERR_ARG (non-positive or
 * non-finite optics, na >= n_medium, even ksize or osr, a non-finite depth, a
 * psf buffer too small); LFRL_ERR_UNSUPPORTED beyond the limits. */
typedef struct {
    double wavelength; /* emission wavelength */
    double na;         /* numerical aperture of the objective */
    double n_medium;   /* refractive index of the immersion medium, > na */
    double mag;        /* objective magnification */
    double d_ml;       /* lenslet pitch (sensor side) */
    double f_ml;       /* lenslet focal length = lenslet-to-sensor distance */
    int32_t nnum;      /* sensor pixels per lenslet per axis (1..64) */
    int32_t nz;        /* depth planes */
    int32_t ksize;     /* PSF window in pixels, odd */
    int32_t osr;       /* field samples per pixel per axis, odd */
    int32_t nquad;     /* quadrature nodes of the Debye integral (0: 1024) */
    uint32_t flags;    /* LFRL_PSF_UNIT_SUM or 0 */
} lfrl_optics;

enum { LFRL_PSF_UNIT_SUM = 1u << 0 };

int lfrl_psf_compute(const lfrl_optics *optics, const double *depths /* [host] nz */,
                     float *psf, void *stream);

/* Kernel timing with HIP events on the caller's stream, for benchmarks.
 * While enabled, every launch of the two spectral contraction kernels is
 * bracketed by events.  lfrl_profile_read synchronises and returns, for
 * kernel "contract_fwd" or "contract_adj", the summed duration in ms and the
 * number of launches since profiling was last enabled. */
int lfrl_profile_enable(lfrl_plan_t plan, int32_t on);
int lfrl_profile_read(lfrl_plan_t plan, const char *kernel, double *total_ms,
                      int64_t *launches);

/* Message describing the last error on this thread ("" if none). */
const char *lfrl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LFRL_H */
