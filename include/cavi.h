/*
 * cavi.h -- C ABI of the MI355X (gfx950) library for the mean-field
 * variational (CAVI) sweep of the Gaussian mixture model of cell
 * subpopulations in qPCR expression data.
 *
 * Model (the mixture reading of the paper's conjugate-exponential framing,
 * Section 3.3; priors of the form of eqs 5-7):
 *   pi ~ Dir(alpha0 1_K);  tau_kg ~ Gamma(a0, rate b0);
 *   mu_kg | tau_kg ~ N(m0_g, 1/(beta0 tau_kg));
 *   z_n ~ Cat(pi);  x_ng | z_n = k ~ N(mu_kg, 1/tau_kg).
 * Variational family (eqs 9 and 13): q = prod_n Cat(z_n | r_n) Dir(pi | alpha)
 *   prod_kg NormalGamma(mu_kg, tau_kg | m_kg, beta_kg, a_kg, b_kg).
 * One sweep (eq 12 applied block by block, Section 3.4):
 *   expectations (eqs 26-31) -> per-row expected log-likelihoods under every
 *   subpopulation -> log-sum-exp responsibilities -> sufficient statistics
 *   (weighted counts, sums and sums of squares per subpopulation and gene)
 *   -> conjugate updates (forms of eqs 16, 17 and 24) -> the lower bound
 *   (eqs 10-11).
 *
 * Conventions
 *   - Every function returns cavi_status; nothing throws across the ABI.
 *     On failure cavi_last_error() (thread-local) holds a message.
 *   - Data X is FP32, row-major N x G, in DEVICE memory, caller-owned; it must
 *     stay alive and unchanged until the handle is destroyed.  The library
 *     never copies or frees it.  It must be 16-byte aligned.
 *   - State arrays passed to set/get are HOST memory, FP64, caller-owned:
 *     alpha[K], and m, beta, a, b as K x G arrays, k-major (index k*G + g).
 *   - All work is enqueued on the stream given at creation (a hipStream_t
 *     passed as void*).  NULL: the handle creates a blocking stream of its
 *     own (sweeps are captured into a hipGraph, which the default stream
 *     cannot hold); work on the default stream is then ordered before and
 *     after the handle's work, work on other streams is not and must be
 *     synchronised by the caller.  Functions that return
 *     results to the host (get_*, sweep with an ELBO buffer, run) synchronise
 *     that stream.  A handle is not thread-safe.
 *   - Workspace: pass device memory of at least cavi_workspace_bytes() bytes
 *     (256-byte aligned), or NULL to let the library allocate (and free on
 *     destroy).
 *   - Determinism: results are bitwise reproducible run to run for the same
 *     inputs, shapes and library build.  The reduction over rows is defined
 *     over fixed 2048-row chunks combined in a fixed order.
 *   - Limits: 1 <= K <= 64, 1 <= G <= 512, K*G <= 4096, K <= N < 2^31.
 */
#ifndef CAVI_H
#define CAVI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CAVI_OK = 0,
    CAVI_E_INVAL = 1,   /* bad argument (shape, pointer, alignment, limit) */
    CAVI_E_NOMEM = 2,   /* workspace too small or allocation failed */
    CAVI_E_HIP = 3,     /* a HIP runtime call failed; message has its text */
    CAVI_E_NUMERIC = 4, /* non-finite statistic or bound; state rolled back */
    CAVI_E_NOTCONV = 5, /* max_sweeps reached without convergence (state valid) */
    CAVI_E_STATE = 6    /* called before a state was initialised or set */
} cavi_status;

typedef struct cavi_ctx cavi_ctx;

/* Prior hyperparameters (eqs 5-7 in mixture form).  m0 is a HOST array of G
 * values, or NULL for the per-gene mean of X (computed on the device). */
typedef struct {
    double alpha0; /* Dirichlet concentration, > 0 */
    double beta0;  /* prior precision scale of the means (q0 of eq 6), > 0 */
    double a0;     /* Gamma shape (eq 5), > 0 */
    double b0;     /* Gamma rate (eq 5), > 0 */
    const double *m0;
} cavi_prior;

/* Defaults: alpha0 = 1 (the Dirichlet(1,1,1) of the synthetic study in
 * Section 4), beta0 = 0.001 and a0 = b0 = 0.5 (the constants of Section 3.5),
 * m0 = NULL. */
cavi_status cavi_prior_default(cavi_prior *prior);

/* Bytes of device workspace needed for one dataset of this shape. */
cavi_status cavi_workspace_bytes(int64_t N, int32_t G, int32_t K, size_t *bytes);

/* Create a handle over device data X (N x G FP32).  prior may be NULL for the
 * defaults.  hip_stream is a hipStream_t or NULL.  workspace_dev may be NULL
 * (library-owned) or caller memory of ws_bytes >= cavi_workspace_bytes().
 * Errors: CAVI_E_INVAL for N < K, G or K out of limits, null out/x_dev,
 * misaligned x_dev, non-positive hyperparameters; CAVI_E_NOMEM for a short
 * workspace; CAVI_E_HIP on a runtime failure. */
cavi_status cavi_create(cavi_ctx **out, const float *x_dev, int64_t N, int32_t G, int32_t K,
                        const cavi_prior *prior, void *hip_stream, void *workspace_dev,
                        size_t ws_bytes);

/* Standard initial state: k-means++ seeds drawn with SplitMix64(seed) from
 * D^2 weights quantised to integers, hard nearest-seed responsibilities, then
 * one conjugate update.  Resets the sweep counter. */
cavi_status cavi_init_standard(cavi_ctx *ctx, uint64_t seed);

/* Inject a state (host FP64 arrays; see Conventions).  Resets the sweep
 * counter.  CAVI_E_INVAL for non-finite or non-positive alpha/beta/a/b. */
cavi_status cavi_set_state(cavi_ctx *ctx, const double *alpha, const double *m,
                           const double *beta, const double *a, const double *b);

/* Copy the current posterior q(pi) q(mu,tau) to host arrays; syncs. */
cavi_status cavi_get_state(cavi_ctx *ctx, double *alpha, double *m, double *beta, double *a,
                           double *b);

/* Run exactly n sweeps (no convergence stop).  elbo_host: NULL, or n doubles
 * receiving the bound after each sweep (then the stream is synchronised).
 * CAVI_E_NUMERIC if a sweep produced a non-finite value: the state is left
 * at the last good sweep. */
cavi_status cavi_sweep(cavi_ctx *ctx, int32_t n, double *elbo_host);

/* Sweep until |L_t - L_{t-1}| <= rel_tol |L_t| (t >= 2 sweeps of this call)
 * or max_sweeps.  sweeps / elbo (may be NULL) receive the number of sweeps
 * run and the final bound.  CAVI_E_NOTCONV when max_sweeps is reached. */
cavi_status cavi_run(cavi_ctx *ctx, int32_t max_sweeps, double rel_tol, int32_t *sweeps,
                     double *elbo);

/* Responsibilities of the current state (the E-step only), written to caller
 * device memory r_dev (N x K FP32, row-major).  Enqueued, not synchronised. */
cavi_status cavi_get_responsibilities(cavi_ctx *ctx, float *r_dev);

/* The per-gene prior centre in use (host array of G doubles). */
cavi_status cavi_get_prior_mean(cavi_ctx *ctx, double *m0_host);

/* Measurement aid: time reps back-to-back launches of the fused E-step +
 * statistics kernel (the sweep's dominant kernel) with HIP events on the
 * handle's stream; *avg_ms receives the mean milliseconds per launch.  Needs
 * a state; rewrites only the per-chunk partials (the state is unchanged).
 * Synchronises the stream. */
cavi_status cavi_profile_estep(cavi_ctx *ctx, int32_t reps, float *avg_ms);

/* Free the handle (and the workspace if library-owned).  NULL is a no-op. */
cavi_status cavi_destroy(cavi_ctx *ctx);

/* Measurement aid (the achievable-read reference of the roofline): a plain
 * streaming read of the n floats at x_dev (device, 16-byte aligned, caller-
 * owned) by grid workgroups of 256 threads with 16-byte loads; out_dev
 * (caller device memory, grid floats) receives per-workgroup sums.  One
 * warm-up launch, then reps launches timed with HIP events on hip_stream
 * (NULL: the null stream); *avg_ms receives the mean milliseconds per launch.
 * Synchronises the stream.  CAVI_E_INVAL for NULL pointers, n, grid or
 * reps < 1, or a misaligned x_dev. */
cavi_status cavi_probe_read(const float *x_dev, int64_t n, float *out_dev, int32_t grid, int32_t reps,
                            void *hip_stream, float *avg_ms);

/* ------------------------------------------------------------------------
 * Batches: B independent datasets sharing G, swept together (one set of
 * launches per sweep, each dataset with its own convergence test).  The same
 * kernels and the same per-dataset reduction order as a single-dataset
 * handle, so a dataset's results are bitwise those of a single handle over
 * its rows when both run the same E-step arithmetic: the E-step is compiled
 * for the handle's largest K, and for G in {16, 32, 48, 64, 96, 128} a
 * largest K up to 8 and one in 9..16 round differently (a dataset with K up
 * to 8 in a batch whose largest K is above 8 agrees with a single handle to
 * rounding, not bitwise).
 *   - x_dev holds the rows of all datasets concatenated (dataset 0 first),
 *     sum(N) x G FP32, device memory, caller-owned, 16-byte aligned.
 *   - N and K are HOST arrays of B entries; each dataset obeys the
 *     single-dataset limits.
 *   - prior->m0, if given, is a HOST array of B x G centres; NULL selects
 *     each dataset's per-gene mean.
 *   - The bound history keeps only the last value per dataset.
 * ------------------------------------------------------------------------ */
typedef struct cavi_batch cavi_batch;

cavi_status cavi_batch_workspace_bytes(int32_t B, const int64_t *N, const int32_t *K, int32_t G,
                                       size_t *bytes);

cavi_status cavi_batch_create(cavi_batch **out, int32_t B, const float *x_dev, const int64_t *N,
                              const int32_t *K, int32_t G, const cavi_prior *prior, void *hip_stream,
                              void *workspace_dev, size_t ws_bytes);

/* Standard initialisation of every dataset on the device; dataset b uses the
 * SplitMix64 state seed + b (the same seeds as cavi_init_standard(seed + b)
 * on a single handle over its rows). */
cavi_status cavi_batch_init_standard(cavi_batch *bt, uint64_t seed);

/* State of dataset b (host arrays sized by its own K; layout as for
 * cavi_set_state).  Coefficients are rebuilt at the next sweep or run. */
cavi_status cavi_batch_set_state(cavi_batch *bt, int32_t b, const double *alpha, const double *m,
                                 const double *beta, const double *a, const double *bb);
/* Learned warm start: every dataset's state from the MLP output rows
 * out_dev (device, FP32, B rows of stride ld >= K(2G+1), dataset order).
 * Row layout [mu' (K x G) | ln E[tau] (K x G) | proportion logits (K)],
 * subpopulation-major, mu = 25 + 10 mu'.  With pi = softmax(logits) and
 * n_k = N pi_k the state is the conjugate posterior those moments give:
 * alpha_k = alpha0 + n_k, beta = beta0 + n_k, m = mu, a = a0 + n_k / 2,
 * b = a / E[tau] (ln E[tau] clamped to [-30, 30]).  The paper has no warm
 * start: this only chooses the starting point of the coordinate updates of
 * Section 3.4, which then run as from any set state.  out_dev must be
 * complete when the handle's stream reaches this call (written on that
 * stream or on the default stream, or synchronised).  Synchronises the
 * stream. */
cavi_status cavi_batch_set_state_warm(cavi_batch *bt, const float *out_dev, int32_t ld);

/* Every dataset's current state as a row (rows_dev: caller device FP32, row
 * b at rows_dev + b*ld) in the layout cavi_batch_set_state_warm reads back:
 * (m - 25)/10 [K*G] | ln(a/b) [K*G] | ln max(alpha - alpha0, 1/2) [K]
 * (alpha - alpha0 are the subpopulation counts N_k, floored at half a row;
 * the softmax of their logs is N_k / N up to the floor), then, when
 * with_centre != 0, the prior centre (m0 - 25)/10 [G].
 * The learned refinement of the standard initialisation reads these rows.
 * Synchronises.  CAVI_E_INVAL for NULL pointers or ld too small; CAVI_E_STATE
 * without a state. */
cavi_status cavi_batch_get_rows(cavi_batch *bt, float *rows_dev, int32_t ld, int32_t with_centre);

cavi_status cavi_batch_get_state(cavi_batch *bt, int32_t b, double *alpha, double *m, double *beta,
                                 double *a, double *bb);

/* Exactly n sweeps of every dataset; synchronises the stream. */
cavi_status cavi_batch_sweep(cavi_batch *bt, int32_t n);

/* Sweep every dataset until its own relative-change test passes (t >= 2
 * sweeps of this call) or max_sweeps.  sweeps / elbo: NULL or B entries;
 * n_converged: NULL or the count of converged datasets.  CAVI_E_NOTCONV
 * when at least one dataset did not converge (all states valid). */
cavi_status cavi_batch_run(cavi_batch *bt, int32_t max_sweeps, double rel_tol, int32_t *sweeps,
                           double *elbo, int32_t *n_converged);

cavi_status cavi_batch_destroy(cavi_batch *bt);

/* ------------------------------------------------------------------------
 * Learned warm start (not in the paper; it only supplies the starting state
 * of the Section 3.4 iteration).  A per-dataset feature vector is mapped by
 * an MLP to a variational state (cavi_batch_set_state_warm).
 *
 * Features (cavi_features): for each dataset b (rows row_off[b] ..
 * row_off[b+1]-1 of the FP32 device array x_dev, G <= 512 columns, row_off a
 * DEVICE int64 array of B+1 offsets) and gene g, 18 values at
 * feat_dev[b*18G + g*18 + j]: j=0 the mean, j=1 ln max(var, 1e-30)
 * (population variance, FP64 sums), j=2..17 16 rank-bin means: the first
 * M = min(N, 4096) rows are ranked by their row sum over genes (FP64, genes
 * in order; ties by row index), bin i holds ranks [floor(iM/16),
 * max(floor((i+1)M/16), floor(iM/16)+1)) and its value is the mean of gene g
 * over those rows.  Means are stored as (v - 25)/10, the log-variance as is.
 * An empty dataset gets NaN features.  Device output, FP32.
 * cavi_features_quantiles: the same layout and moments, with j=2..17 the 16
 * nearest-rank quantiles of gene g over all N rows instead of the rank bins:
 * sorted(x_g)[floor((i + 0.5) N / 16)], i = 0..15 (the per-gene summary of
 * the warm-start workload), stored as (v - 25)/10.
 *
 * Targets (cavi_warm_targets): from generating parameters (DEVICE FP64:
 * pi[B*K], mu[B*K*G], tau[B*K*G], k-major per dataset) the training target
 * rows target_dev[b*K(2G+1) ..]: subpopulations ordered by their mean over
 * genes (ascending, ties by index), then [(mu-25)/10 | ln tau | ln pi].
 *
 * MLP (cavi_mlp_*): in_dim -> hidden (x n_hidden, exact-erf GELU) -> out_dim
 * linear.  FP32 master parameters, for each layer l: W_l (out x in,
 * row-major) then b_l, concatenated; initialised W ~ U(-1/sqrt(in),
 * 1/sqrt(in)) from SplitMix64(seed), b = 0.  Every product rounds both
 * operands to BF16 (round to nearest even) and accumulates in FP32 on the
 * matrix cores; bias, activation, loss and optimiser are FP32.
 *   forward:   out_dev[B x out_dim] for feat_dev[B x in_dim] (device).
 *   loss_grad: forward, loss = mean over B*out_dim of (y - t)^2, gradients
 *              of that loss into the library's gradient buffer (overwritten);
 *              loss_host (may be NULL) receives the loss (synchronises).
 *   adamw:     one AdamW step (decoupled weight decay, bias-corrected
 *              moments, step count kept by the handle).
 *   get/set_params, get_grads: HOST FP32 arrays of n_params entries
 *              (synchronise).
 *   get_layer: HOST copy (B x dims[layer], row-major FP32; synchronises) of
 *              what the last call left for linear layer `layer` (1 .. n_hidden
 *              + 1): what = 0 its pre-activation Z (forward, loss_grad), 1 its
 *              output Y (for the last layer only after loss_grad, since
 *              forward writes it to out_dev), 2 the loss gradient w.r.t. Z
 *              (loss_grad).  Lets each product be checked with the operands
 *              it was given.
 * B <= max_batch.  Work is enqueued on hip_stream (NULL: the default
 * stream, so that outputs are ordered before a CAVI handle's later work).
 * Not thread-safe.
 * ------------------------------------------------------------------------ */
cavi_status cavi_features(const float *x_dev, const int64_t *row_off_dev, int32_t B, int32_t G,
                          float *feat_dev, void *hip_stream);
cavi_status cavi_features_quantiles(const float *x_dev, const int64_t *row_off_dev, int32_t B, int32_t G,
                                    float *feat_dev, void *hip_stream);
cavi_status cavi_warm_targets(const double *pi_dev, const double *mu_dev, const double *tau_dev,
                              int32_t B, int32_t K, int32_t G, float *target_dev, void *hip_stream);
/* y[i*ldy + j] += alpha * x[i*ldx + j] for i < n, j < m (device FP32 arrays,
 * caller-owned; enqueued on hip_stream).  The refinement's targets (converged
 * rows minus initial rows) and its output (initial rows plus the network's
 * move) are formed with it.  CAVI_E_INVAL for NULL pointers, n or m < 1, or
 * strides below m. */
cavi_status cavi_rows_axpy(int32_t n, int32_t m, float alpha, const float *x_dev, int32_t ldx, float *y_dev,
                           int32_t ldy, void *hip_stream);

typedef struct cavi_mlp cavi_mlp;

cavi_status cavi_mlp_create(cavi_mlp **out, int32_t in_dim, int32_t hidden, int32_t n_hidden,
                            int32_t out_dim, int32_t max_batch, uint64_t seed, void *hip_stream);
cavi_status cavi_mlp_n_params(cavi_mlp *net, int64_t *n);
cavi_status cavi_mlp_get_params(cavi_mlp *net, float *host);
cavi_status cavi_mlp_set_params(cavi_mlp *net, const float *host);
cavi_status cavi_mlp_get_grads(cavi_mlp *net, float *host);
cavi_status cavi_mlp_forward(cavi_mlp *net, const float *feat_dev, int32_t B, float *out_dev);
cavi_status cavi_mlp_loss_grad(cavi_mlp *net, const float *feat_dev, const float *target_dev, int32_t B,
                               float *loss_host);
cavi_status cavi_mlp_get_layer(cavi_mlp *net, int32_t layer, int32_t what, int32_t B, float *host);
cavi_status cavi_mlp_adamw(cavi_mlp *net, float lr, float beta1, float beta2, float eps,
                           float weight_decay);
cavi_status cavi_mlp_destroy(cavi_mlp *net);

/* ------------------------------------------------------------------------
 * E-step schedule (autotuner).  For the shapes of the tiled E-step (G in
 * {16, 32, 48, 64, 96, 128}, K <= 16) two schedules give bitwise the same
 * results: 0 keeps the exact-term loads, centres and responsibilities in
 * registers; 1 keeps them in LDS and needs fewer registers (more waves per
 * SIMD).  At the first sweep, run or profile call the library times both on
 * the handle's data and keeps the faster one; cavi_*set_schedule forces one
 * (-1: tune again at the next call).  ms (NULL or 2 entries) receives the
 * measured average E-step times of schedules 0 and 1 (0 if not measured).
 * ------------------------------------------------------------------------ */
cavi_status cavi_get_schedule(cavi_ctx *ctx, int32_t *schedule, float *ms);
cavi_status cavi_set_schedule(cavi_ctx *ctx, int32_t schedule);
cavi_status cavi_batch_get_schedule(cavi_batch *bt, int32_t *schedule, float *ms);
cavi_status cavi_batch_set_schedule(cavi_batch *bt, int32_t schedule);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (tight serving loops, code
 * run where hipMalloc is not allowed): one dataset fitted without a handle or
 * a workspace.  Standard initialisation (seed), then sweeps until
 * |L_t - L_{t-1}| <= rel_tol |L_t| or max_sweeps, then the state copied to
 * the caller's host arrays (alpha: K; m, beta, a, b: K x G, k-major) and
 * *sweeps / *elbo (may be NULL) set as by cavi_run.  Every device buffer is
 * carved from one static array of cavi_static_scratch_bytes() (64 MiB) that
 * each GPU the library runs on holds until the process ends; the call makes
 * no hipMalloc, hipFree or other allocating call.  x_dev (N x G FP32
 * row-major, 16-byte aligned) is caller-owned and read only.  Work runs on
 * hip_stream (NULL: the null stream) and the call returns when it is done.
 * All calls on one GPU share its array: calls that overlap on one GPU (other
 * threads, other streams) race and must be serialised by the caller.  Same
 * kernels, order and results as cavi_create + cavi_init_standard + cavi_run
 * + cavi_get_state.  Errors as those calls, and CAVI_E_NOMEM when N, G and K
 * need more scratch than the array holds (the message gives both sizes).
 * ------------------------------------------------------------------------ */
size_t cavi_static_scratch_bytes(void);
cavi_status cavi_fit_static(const float *x_dev, int64_t N, int32_t G, int32_t K, const cavi_prior *prior,
                            uint64_t seed, int32_t max_sweeps, double rel_tol, void *hip_stream,
                            double *alpha, double *m, double *beta, double *a, double *b,
                            int32_t *sweeps, double *elbo);

/* Thread-local text of the last error ("" if none). */
const char *cavi_last_error(void);

/* Library version string. */
const char *cavi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CAVI_H */
