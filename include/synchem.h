/*
 * synchem.h - C ABI of libsynchem: the EM iteration of Synch-EM for 2-D multi-reference
 * alignment (Janco & Bendory, "An accelerated expectation-maximization algorithm for
 * multi-reference alignment"), on one AMD Instinct MI355X (gfx950).
 *
 * Model (Section I, eq. (4)): observation j is v_j = a o exp(-i kbar theta_j) + eps_j, with a the
 * D = K*Q steerable coefficients of the image (k-major: entry d = k*Q + q has angular index
 * kbar[d] = d / Q), theta_j on the grid 2*pi*l/L, and eps_j circular complex Gaussian with
 * E|eps_jd|^2 = sigma2.  The EM (Section II-B, eqs. (14)-(18); Algorithm "Synch-EM") visits the
 * rotation offsets o_i = window_lo + i, i = 0..window_count-1 (Section III-C); plain EM over all
 * rotations is window_lo = 0, window_count = L.  rho has one entry per visited offset.
 *
 * Conventions for every entry point:
 *  - Complex vectors are interleaved (re, im) doubles or floats, row-major, one row per
 *    observation.  "host" pointers are read or written before the call returns; "device"
 *    pointers must be device memory of the GPU that was current at em_init.
 *  - All device work is enqueued on the context's HIP stream (given at em_init, changed with
 *    em_set_stream).  Calls that return a host value synchronise that stream before returning.
 *  - A context is not thread-safe: calls on one context must not overlap.
 *  - Arguments are validated before any device work; a rejected call returns EM_EINVAL (or
 *    EM_EUNSUPPORTED) and leaves the context unchanged and usable.  em_last_error(ctx) then
 *    describes the problem; em_last_error(NULL) describes the last failure of em_init or
 *    em_learn_prior on the calling thread.
 *  - EM_EDEVICE means a HIP runtime call failed; the context should then be destroyed.
 */
#ifndef SYNCHEM_H
#define SYNCHEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct em_ctx em_ctx;              /* opaque, owned by the library */

typedef enum {
    EM_OK = 0,
    EM_EINVAL = -1,          /* invalid argument (nothing was done)                        */
    EM_ENOMEM = -2,          /* device allocation failed                                    */
    EM_EDEVICE = -3,         /* a HIP runtime call failed                                   */
    EM_ESTATE = -4,          /* call not valid in the context's state (e.g. bwd before fwd) */
    EM_ENONFINITE = -5,      /* the observations contain NaN or Inf                         */
    EM_EUNSUPPORTED = -6     /* valid but outside the library's limits (see em_params)      */
} em_status;

/* Arithmetic of the observation x template correlation (the E-step contraction).  Every mode
 * reduces across observations in FP64 and assembles the log-likelihood and the M-step in FP64.
 *  EM_FP64   complex128 input, FP64 everywhere.
 *  EM_FP32   complex64 input, FP32 matrix cores (MFMA), FP32 accumulation.
 *  EM_BF16X3 complex64 input, observations and template each split into bf16 hi + lo after a
 *            per-observation power-of-two scaling; three bf16 MFMA products (hi*hi + hi*lo +
 *            lo*hi) accumulated in FP32.
 *  EM_FP16   complex64 input, observations in fp16 after per-observation power-of-two scaling,
 *            template split fp16 hi + lo; two fp16 MFMA products accumulated in FP32.
 *  EM_BF16   as EM_FP16 with bf16 observations (one plane) and a bf16 hi + lo template.       */
typedef enum { EM_FP64 = 0, EM_FP32 = 1, EM_BF16X3 = 2, EM_FP16 = 3, EM_BF16 = 4 } em_precision;

/* flags */
#define EM_FLAG_KEEP_LSE  (1ull << 0)   /* em_step also stores the per-observation log-likelihood
                                           (in the buffer the adjoint checkpoints into, so an
                                           em_step with this flag voids the last em_loglik_fwd) */
#define EM_FLAG_TIMING    (1ull << 1)   /* time every E+M pass with HIP events (em_pass_time)     */
#define EM_FLAG_GENERAL_PASS (1ull << 2) /* use the general pass (template streamed from L2, row
                                           tiles in LDS) instead of the specialised correlation
                                           passes (register-resident template; the FP32 GEMM with
                                           its posterior / M-step epilogue) */
#define EM_FLAG_WIDE_PASS (1ull << 3)   /* EM_FP16 / EM_BF16: always use the wide-row pass variant
                                           (chosen by itself when a row tile does not fit in LDS) */
#define EM_FLAG_FACTORED  (1ull << 4)   /* evaluate the correlations through the per-frequency sums
                                           c_jk = sum_q conj(v_jkq) a_kq (an exact rewrite, by eq.
                                           (3), that needs no template); D = 512 with Q a power-
                                           of-two multiple of 8 (any precision but EM_FP64), or
                                           D = 2048 in EM_FP16 / EM_BF16 with Q a power-of-two
                                           multiple of 16; else EM_EUNSUPPORTED */
#define EM_FLAG_STAGED_PASS (1ull << 5) /* EM_FP16 / EM_BF16 with D = 512: use the pass that stages
                                           whole row tiles in LDS instead of the row-stream pass
                                           (both are the correlation GEMM; for comparisons) */

typedef struct {
    int64_t n_obs;          /* N >= 1                                                        */
    int32_t K, Q;           /* angular x radial sizes, D = K*Q in [1, 2048]; EM_FP64, EM_FP32
                               and EM_BF16X3 need D <= 512 (EM_EUNSUPPORTED above)         */
    int32_t L;              /* rotation grid size >= 1                                        */
    int32_t window_lo;      /* first offset (any integer; taken mod L); 0 when angles is set   */
    int32_t window_count;   /* W in [1, min(L, 1024)]; with angles: W in [1, 1024]            */
    double  sigma2;         /* noise variance per complex entry, > 0                          */
    double  gamma;          /* weight of the KL prior on rho (Section III-B eq. (23)), >= 0   */
    int32_t update_rho;     /* 1: update rho each iteration (eq. (18) / the KL-prior update of
                               Algorithm "Synch-EM"); 0: keep rho fixed                        */
    int32_t precision;      /* em_precision                                                   */
    uint64_t flags;         /* EM_FLAG_*                                                      */
    const double *gamma_a_inv;  /* host, D entries >= 0: diagonal of Gamma_a^{-1}, the inverse
                                   covariance of the Gaussian image prior of eq. (17); NULL: none */
    const double *a0;       /* host, 2D doubles: initial estimate; NULL: the mean of the
                               observations (Algorithm "Synch-EM", initialisation)               */
    const double *angles;   /* host, W finite angles in radians: the rotations searched, in place
                               of the grid offsets window_lo .. window_lo + W - 1 (the refined-
                               resolution window of Section III-C: the likely range sampled more
                               densely than the grid 2 pi / L).  The E-step, the M-step (eq. (17)
                               with exp(+i k theta_i)) and rho (one entry per angle) use these
                               angles; L still sets the grid of the stopping metric.  NULL: the
                               grid window.                                                     */
} em_params;

/* Create a context and load the observations (Algorithm "Synch-EM", inputs and initialisation).
 *  obs_dev  device, N x D complex, row-major: complex128 for EM_FP64, complex64 otherwise.  It is
 *           converted into library-owned storage and not referenced after the call returns.
 *  prior    host, W entries >= 0 with positive sum: the learned distribution rho_bar over the
 *           window (Section III-B); it is normalised to sum 1 and used both as rho_0 and in the
 *           KL-prior update.  NULL: uniform.
 *  stream   hipStream_t (NULL: the null stream).
 * Synchronises the stream.  Returns EM_ENONFINITE if any observation entry is NaN or Inf. */
em_status em_init(em_ctx **out, const em_params *p, const void *obs_dev, const double *prior,
                  void *stream);

/* Run up to n_iter >= 0 EM iterations (Algorithm "Synch-EM" loop: E-step weights over the window
 * (eq. (15)), normalisation, W_t, coefficient update (eq. (17)), distribution update (eq. (18) or
 * the KL-prior update of App. C eq. (42))).  With tol > 0 it stops after the first iteration whose
 * stopping metric min_l ||a_{t+1} - exp(-2 pi i kbar l / L) o a_t||^2 falls below tol; once stopped,
 * further calls do nothing until em_set_state.  iters_done (host, may be NULL) receives the number
 * of iterations performed; ll_last (host, may be NULL) the marginal log-likelihood of the state the
 * last performed iteration started from.  Synchronises the stream when either pointer is given. */
em_status em_step(em_ctx *ctx, int32_t n_iter, double tol, int32_t *iters_done, double *ll_last);

/* Marginal log-likelihood log p(v | a_t, rho_t) of the current state (eq. (13) with the rotation
 * summed over the window), FP64, into *ll (host).  Synchronises. */
em_status em_loglik(em_ctx *ctx, double *ll);

/* Posterior weights of observations [row0, row0 + nrows) at the current state (eq. (15)).
 *  w_dev       device, nrows x W floats, or NULL
 *  argmax_dev  device, nrows int32: most probable window index (lowest index on ties), or NULL
 *  margin_dev  device, nrows floats: best minus runner-up posterior (W = 1: the best), or NULL
 * Asynchronous. */
em_status em_posterior(em_ctx *ctx, int64_t row0, int64_t nrows, float *w_dev,
                       int32_t *argmax_dev, float *margin_dev);

/* Copy the state out (host buffers: a 2D doubles, rho W doubles, t = iterations done; any may be
 * NULL) or in.  em_set_state clears the stop flag.  Synchronises. */
em_status em_get_state(em_ctx *ctx, double *a, double *rho, int64_t *t);
em_status em_set_state(em_ctx *ctx, const double *a, const double *rho, int64_t t);

/* Differentiable marginal log-likelihood LL(a, sigma2, eta) = sum_j log sum_i rho_i
 * p(v_j | o_i, a, sigma2), rho = softmax(eta) (gradients are derived from eq. (13) by the Fisher
 * identity).  The forward pass keeps one FP64 log-likelihood per observation as the checkpoint;
 * the backward pass recomputes the posteriors from it instead of storing N x W weights.
 *  a_dev    device, 2D doubles (complex128); eta_dev device, W doubles, or NULL for the
 *           context's current rho.  *ll (host) receives LL.  Synchronises.
 * em_loglik_bwd(g): gradients of g * LL at the last forward's inputs.
 *  grad_a_dev   device, 2D doubles: dLL/dRe a + i dLL/dIm a, i.e. (2/sigma2) (S - N a)
 *  grad_sigma2  host: -N D / sigma2 + sum_ji w_ji ||R_i a - v_j||^2 / sigma2^2
 *  grad_eta_dev device, W doubles: W_t - N rho, or NULL
 * Returns EM_ESTATE without a preceding successful forward, or when em_set_state or an em_step
 * of a context made with EM_FLAG_KEEP_LSE ran after it (the checkpoint no longer matches the
 * forward's inputs; run the forward again).  Synchronises. */
em_status em_loglik_fwd(em_ctx *ctx, const double *a_dev, double sigma2, const double *eta_dev,
                        double *ll);
em_status em_loglik_bwd(em_ctx *ctx, double g, double *grad_a_dev, double *grad_sigma2,
                        double *grad_eta_dev);

/* Per-iteration statistics, oldest first, EM_STATS_FIELDS doubles per record:
 * t, log-likelihood of the starting state, MAP objective (log-likelihood + gamma sum rho_bar log
 * rho - sum gamma_a^{-1} |a|^2), ||a_{t+1} - a_t||^2, stopping metric, entropy of rho_{t+1}.
 * Keeps the last 1024 iterations.  buf (host) holds cap records; *n receives the count copied. */
#define EM_STATS_FIELDS 6
em_status em_get_stats(em_ctx *ctx, double *buf, int32_t cap, int32_t *n);

/* Learned rotation prior (Section III-B eq. (22); Algorithm "learning rotation distribution"):
 * histogram of n integer rotation errors (device int32, each taken mod L), restricted to the
 * window offsets lo..lo+W-1 and normalised over it.  rho_bar (host, W doubles) receives it;
 * counts (host, L int64, indexed by error mod L, or NULL) the full histogram; *n_in_window (host,
 * or NULL) the number of draws inside the window.  Returns EM_EINVAL if none falls inside.
 * Runs on stream and synchronises it. */
em_status em_learn_prior(const int32_t *err_dev, int64_t n, int32_t L, int32_t lo, int32_t W,
                         double *rho_bar, int64_t *counts, int64_t *n_in_window, void *stream);

/* ---- Synchronize and Match: the step before the EM path (§II-A, §III-A).
 * These calls take the caller's observations directly (device, N x D complex64, row-major, the
 * same layout as em_init; not copied), run on stream and synchronise it, allocate their own
 * scratch and free it before returning.  They return EM_EINVAL for a missing pointer or a size
 * out of range (before any device work), EM_EUNSUPPORTED beyond the stated limits, EM_ENOMEM
 * when scratch cannot be allocated, EM_EDEVICE for a failed HIP call; em_last_error(NULL)
 * describes the failure.
 * Observations must be finite (not checked here; em_init checks them).  Ties in an argmax or
 * argmin go to the lowest index.  Sign conventions: R_l v = v o exp(-i kbar 2 pi l / L); rel[i][j]
 * is the grid rotation that best maps v_j onto v_i, an estimate of theta_i - theta_j; the
 * alignment multiplies by exp(+i kbar theta_i). */

/* Relative rotations between all pairs of the first P observations (§II-A, the pairwise
 * estimate): rel[i*P + j] = argmax_l Re <v_i, R_l v_j> over l = 0..L-1, computed through the
 * per-frequency sums c_ijk = sum_q conj(v_ikq) v_jkq and FP32 matrix cores.  Optional outputs
 * (device, P x P, may be NULL): gap = the best correlation minus the runner-up, dot = Re <v_i, v_j>
 * (the l = 0 correlation).  2 <= P <= 8192, 1 <= L <= 4096, D <= 2048, K <= 512. */
em_status em_relative_rotations(const void *obs_dev, int64_t P, int32_t K, int32_t Q, int32_t L,
                                int32_t *rel_dev, float *gap_dev, float *dot_dev, void *stream);

/* Projected power method of angular synchronization (§II-A): from z = 1, iters times
 * z <- phase(H z) with H_ij = exp(+i 2 pi rel_ij / L) (FP64; an entry with H z = 0 keeps its
 * value); theta_dev (device, P doubles) = arg z in [-pi, pi]. */
em_status em_ppm(const int32_t *rel_dev, int64_t P, int32_t L, int32_t iters, double *theta_dev,
                 void *stream);

/* Nearest neighbours (Algorithm "Synchronize and Match", the matching step): for every
 * observation i < N the member n of S_P = {0 .. P-1}, n != i, minimising ||v_i - v_n||^2 (no
 * rotation; FP32 matrix cores).  nn_dev: N int32; gap_dev (N floats or NULL): the runner-up's
 * squared distance minus the best.  2 <= P <= N; D a multiple of 8. */
em_status em_nearest(const void *obs_dev, int64_t N, int32_t K, int32_t Q, int64_t P,
                     int32_t *nn_dev, float *gap_dev, void *stream);

/* Algorithm "Synchronize and Match": relative rotations and the power method (iters iterations)
 * on S_P = the first P observations, then theta_i = phi_{nn_i} for every observation.
 * theta_dev: N doubles (radians); nn_dev: N int32 or NULL. */
em_status em_sync_match(const void *obs_dev, int64_t N, int32_t K, int32_t Q, int32_t L,
                        int64_t P, int32_t iters, double *theta_dev, int32_t *nn_dev,
                        void *stream);

/* Aligned observations (§II-A): out[i] = v_i o exp(+i kbar theta_i), complex64, N x D (device,
 * caller-owned, must not overlap obs_dev). */
em_status em_align(const void *obs_dev, int64_t N, int32_t K, int32_t Q, const double *theta_dev,
                   void *out_dev, void *stream);

/* The average of the aligned coefficients (§II-A): mean_dev (device, 2D doubles, re/im
 * interleaved) = (1/N) sum_i v_i o exp(+i kbar theta_i), FP64 with FP64 phases, fixed-order
 * sums.  After Synchronize and Match it is the EM's starting point (§III-A); in the algorithm that
 * learns the rotation distribution it gives the global rotation theta_c. */
em_status em_aligned_mean(const void *obs_dev, int64_t N, int32_t K, int32_t Q,
                          const double *theta_dev, double *mean_dev, void *stream);

/* em_aligned_mean for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same arguments, the same kernels and
 * the same result bit for bit, but no hipMalloc, hipFree or allocating library call.  Its
 * partial sums live in the library's own static device array of 8 MiB per GPU (256 x 2 x 2048
 * doubles, held until the process ends), which covers every D the library accepts (D <= 2048;
 * larger shapes are rejected with EM_EUNSUPPORTED before any device work).  The work is enqueued
 * on `stream` and the call returns without waiting: mean_dev is ready in stream order.  All calls
 * on one GPU share that array, so calls that overlap on one GPU (on different streams, or from
 * several threads) race and must be serialised by the caller.  Errors as em_aligned_mean
 * (em_last_error(NULL)); a failure to look up the array's address returns EM_EDEVICE. */
em_status em_aligned_mean_noalloc(const void *obs_dev, int64_t N, int32_t K, int32_t Q,
                                  const double *theta_dev, double *mean_dev, void *stream);

/* Binned centred errors of a synchronizer (§III-B, Algorithm "learning rotation distribution"):
 * bins_dev[i] = floor((theta_hat_i - theta_i - 2 pi lc / L) L / (2 pi)) mod L (FP64), for
 * em_learn_prior.  theta_hat_dev, theta_dev: N doubles (radians); lc: the centring rotation on
 * the grid (em_relative_rotations of the true image and the aligned mean gives it).  After
 * alignment the windowed EM's rotation variable is the negated error: its prior is the histogram
 * of the bins computed with the two angle arrays swapped and -lc. */
em_status em_error_bins(const double *theta_hat_dev, const double *theta_dev, int64_t N, int32_t L,
                        int32_t lc, int32_t *bins_dev, void *stream);

/* Change the stream of later calls. */
em_status em_set_stream(em_ctx *ctx, void *stream);

/* With EM_FLAG_TIMING: total milliseconds and number of timed E+M passes since the last reset
 * (reset != 0 clears them after reading).  Synchronises. */
em_status em_pass_time(em_ctx *ctx, double *ms_total, int64_t *launches, int32_t reset);

/* Launch geometry and storage of the context (for reports): rows per tile, workgroups of the E+M
 * pass, bytes of observation storage per row, padded window, name of the E+M kernel variant that
 * em_step runs (posterior queries and the adjoint's passes of a factored context over a window
 * symmetric about 0 run the plain factored variant). */
typedef struct {
    int32_t rows_per_tile, grid, threads, window_padded;
    int64_t bytes_per_row;
    int64_t lds_bytes;
    char kernel[64];
} em_info;
em_status em_get_info(const em_ctx *ctx, em_info *info);

void em_destroy(em_ctx *ctx);
const char *em_last_error(const em_ctx *ctx);
const char *em_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SYNCHEM_H */
