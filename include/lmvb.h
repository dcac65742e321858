/*
 * lmvb.h -- C ABI of the gfx950 variational Bayes for the paper's own linear-mixing model of a
 * heterogeneous tissue (Section 3.3, eqs 2-8; updates eqs 16-31; steps of Section 3.5).
 *
 * Model.  V genes, N subpopulations (Boolean networks), M = N - 1.  Gene i has one reading r_i
 * and an expression profile d_i (N values); mu_i = d_{i,N}, D_i = (d_{i,q} - d_{i,N})_{q<N}:
 *   r_i ~ N(D_i^T beta_i + mu_i, 1/rho)        (eq 3)
 *   beta_i ~ N(K, Lambda^-1)                   (eq 4; beta_i are the gene's first M weights)
 *   rho ~ Gamma(a0, rate b0)                   (eq 5)
 *   K | Lambda ~ N(K0, (q0 Lambda)^-1)         (eq 6)
 *   Lambda ~ Wishart(n0 degrees of freedom, scale L0), E[Lambda] = n0 L0   (eq 7)
 * Variational family (eq 13): q(rho) = Gamma(a_rho, b_rho); q(beta_i) = N(m_i, P_i^-1);
 *   q(K, Lambda) = N(K | K0K, (kappa Lambda)^-1) Wishart(Lambda | nu, scale W) with
 *   kappa = q0 + V, nu = n0 + V; W is the paper's Lambda_0Lambda (E[Lambda] = nu W, eq 28).
 * One sweep (Section 3.5, steps 1-6): q(rho) from the current q(beta) (eqs 16, 17); q(beta_i) for
 *   every gene (eqs 20, 21 with eqs 28, 29, 31); q(K, Lambda) from the new q(beta) (eqs 24, 25 with
 *   eqs 26, 27); then the lower bound (eq 11, written out in full; the Wishart prior's
 *   normalising constant is left out when the prior is improper, n0 <= M - 1).
 *
 * Conventions (as in cavi.h; the status codes and cavi_last_error() are shared):
 *   - r (V) and d (V x N, row-major) are FP64 in DEVICE memory, caller-owned, 8-byte aligned,
 *     unchanged and alive until the handle is destroyed.  The library never copies or frees them.
 *   - Host arrays are FP64 and caller-owned; matrices are M x M row-major.
 *   - Work runs on the stream given at creation (hipStream_t as void*; NULL: a blocking stream of
 *     the handle's own).  Functions returning results to the host synchronise it.  A handle is not
 *     thread-safe.  The library allocates its own device memory (O(V / 256) doubles at most).
 *   - Determinism: results are bitwise reproducible run to run; sums over genes are defined over
 *     chunks of 256 p consecutive genes, p = min(32, max(1, ceil(V / 2^18))), combined in a fixed
 *     order.
 *   - Limits: 1 <= V < 2^40, 2 <= N <= 8, n0 + V > N - 2.
 */
#ifndef LMVB_H
#define LMVB_H

#include <stddef.h>
#include <stdint.h>

#include "cavi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lmvb_ctx lmvb_ctx;

/* Prior constants (Section 3.5).  K0 (M values) and L0 (M x M, symmetric positive definite, the
 * prior scale matrix of Lambda) are host arrays read at creation. */
typedef struct {
    double a0, b0, q0, n0;
    const double *K0;
    const double *L0;
} lmvb_prior;

/* Create a handle over r_dev (V) and d_dev (V x N).  prior NULL: the paper's constants: a0 = b0 =
 * 0.5, q0 = 0.001, n0 = 1, K0 = 1/N, L0 = [[0.01, 0.005], [0.005, 0.008]]^-1 for N = 3 and 100 I
 * otherwise.  CAVI_E_INVAL: bad shape, NULL or misaligned pointer, non-finite or non-positive
 * constant, L0 not positive definite.  The state is undefined until lmvb_init. */
cavi_status lmvb_create(lmvb_ctx **out, const double *r_dev, const double *d_dev, int64_t V, int32_t N,
                        const lmvb_prior *prior, void *hip_stream);

/* The initial state of Section 3.5: P_i = L0, m_i = K0K = 1/N, a_rho = a0, b_rho = b0 and the
 * matrix of eq 25 set to L0 (W = L0^-1); one pass over the genes forms the bracket of eq 17 under
 * this q(beta).  Synchronises.  CAVI_E_NUMERIC if that statistic is not finite. */
cavi_status lmvb_init(lmvb_ctx *h);

/* n >= 1 sweeps.  elbo_host: NULL or n values, the bound after each sweep.  Synchronises.
 * CAVI_E_STATE before lmvb_init; CAVI_E_NUMERIC if a sweep produced a non-finite value (the
 * globals keep the last finite state). */
cavi_status lmvb_sweep(lmvb_ctx *h, int32_t n, double *elbo_host);

/* Sweeps until |L_t - L_{t-1}| <= rel_tol |L_t| (t >= 2 within the call) or max_sweeps.
 * sweeps, elbo: NULL or outputs.  CAVI_E_NOTCONV when max_sweeps is reached (state valid). */
cavi_status lmvb_run(lmvb_ctx *h, int32_t max_sweeps, double rel_tol, int32_t *sweeps, double *elbo);

/* The global factors: a_rho, b_rho, K0K (M), W (M x M), nu, kappa.  Any pointer may be NULL. */
cavi_status lmvb_get_globals(lmvb_ctx *h, double *a_rho, double *b_rho, double *K0K, double *W, double *nu,
                             double *kappa);

/* The gene factors of the current state into DEVICE arrays (either may be NULL): m_dev (V x M) and
 * P_dev (V x M x M).  Enqueued on the handle's stream; synchronises. */
cavi_status lmvb_get_genes(lmvb_ctx *h, double *m_dev, double *P_dev);

/* Average duration (ms, HIP events on the handle's stream) of reps launches of the per-gene pass
 * with the current coefficients (the state is unchanged).  Synchronises. */
cavi_status lmvb_profile_pass(lmvb_ctx *h, int32_t reps, float *ms);

/* Release the handle (NULL is a no-op). */
cavi_status lmvb_destroy(lmvb_ctx *h);

#ifdef __cplusplus
}
#endif

#endif /* LMVB_H */
