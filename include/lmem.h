/*
 * lmem.h -- C ABI of the gfx950 expectation maximisation for the paper's linear-mixing model of a
 * heterogeneous tissue (Section 3.3, eqs 3 and 4; iteration of Section 4.2, eqs 42-47).
 *
 * Model.  V genes, N subpopulations, M = N - 1.  Gene i has one reading r_i and an expression
 * profile d_i (N values); mu_i = d_{i,N}, D_i = (d_{i,q} - d_{i,N})_{q<N}:
 *   r_i ~ N(D_i^T beta_i + mu_i, 1/rho)   (eq 3)
 *   beta_i ~ N(K, Lambda^-1)              (eq 4)
 * EM estimates rho, K and Lambda with the beta_i as hidden variables.  One iteration from the
 * estimates (rho, K, Lambda):
 *   E-step, every gene: Sigma_i = (Lambda + rho D_i D_i^T)^-1 (eq 42),
 *     M_i = Sigma_i (Lambda K + rho D_i (r_i - mu_i)) (eq 43), S_i (eq 44);
 *   M-step: rho = V / sum S_i (eq 45), K = sum M_i / V (eq 46),
 *     Lambda^-1 = sum (M_i M_i^T + Sigma_i) / V - K K^T (eq 47).
 * Each iteration also yields the marginal log-likelihood of the estimates it started from,
 *   sum_i ln N(r_i; mu_i + D_i^T K, 1/rho + D_i^T Lambda^-1 D_i),
 * the quantity EM never decreases, used for the stopping test.
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
 *   - Limits: 1 <= V < 2^40, 2 <= N <= 8.
 */
#ifndef LMEM_H
#define LMEM_H

#include <stddef.h>
#include <stdint.h>

#include "cavi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lmem_ctx lmem_ctx;

/* Starting estimates: rho > 0, K (M values), Lambda (M x M, symmetric positive definite); host
 * arrays read at creation. */
typedef struct {
    double rho;
    const double *K;
    const double *Lam;
} lmem_start;

/* Create a handle over r_dev (V) and d_dev (V x N), at the starting estimates.  start NULL: the
 * means of the paper's priors (eqs 5-7 with the constants of Section 3.5): rho = a0 / b0 = 1,
 * K = 1/N, Lambda = n0 L0 = [[0.01, 0.005], [0.005, 0.008]]^-1 for N = 3 and 100 I otherwise.
 * CAVI_E_INVAL: bad shape, NULL or misaligned pointer, rho not finite and positive, K not finite,
 * Lambda not symmetric positive definite. */
cavi_status lmem_create(lmem_ctx **out, const double *r_dev, const double *d_dev, int64_t V, int32_t N,
                        const lmem_start *start, void *hip_stream);

/* n >= 1 iterations.  loglik_host: NULL or n values, the log-likelihood of the estimates each
 * iteration started from.  Synchronises.  CAVI_E_NUMERIC if an iteration produced a non-finite
 * value or a Lambda^-1 that is not positive definite (the estimates keep the last valid ones). */
cavi_status lmem_iterate(lmem_ctx *h, int32_t n, double *loglik_host);

/* Iterations until |l_t - l_{t-1}| <= rel_tol |l_t| for the log-likelihoods l_t of two successive
 * iterations of this call (the iteration that finds it is completed), or max_iter.
 * iters, loglik: NULL or outputs (the last l_t).  CAVI_E_NOTCONV when max_iter is reached
 * (estimates valid). */
cavi_status lmem_run(lmem_ctx *h, int32_t max_iter, double rel_tol, int32_t *iters, double *loglik);

/* The current estimates: rho, K (M), Lambda (M x M) and Lambda^-1 (M x M, as eq 47 forms it).
 * Any pointer may be NULL. */
cavi_status lmem_get_params(lmem_ctx *h, double *rho, double *K, double *Lam, double *Laminv);

/* The E-step of the current estimates into DEVICE arrays (either may be NULL): M_dev (V x M,
 * eq 43) and Sigma_dev (V x M x M, eq 42).  Enqueued on the handle's stream; synchronises. */
cavi_status lmem_get_genes(lmem_ctx *h, double *M_dev, double *Sigma_dev);

/* Average duration (ms, HIP events on the handle's stream) of reps launches of the per-gene E-step
 * pass at the current estimates (the estimates are unchanged).  Synchronises. */
cavi_status lmem_profile_pass(lmem_ctx *h, int32_t reps, float *ms);

/* Release the handle (NULL is a no-op). */
cavi_status lmem_destroy(lmem_ctx *h);

#ifdef __cplusplus
}
#endif

#endif /* LMEM_H */
