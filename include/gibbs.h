/*
 * gibbs.h -- C ABI of the gfx950 Gibbs sampler for the paper's linear-mixing model of a
 * heterogeneous tissue (Section 3.3, eqs 3-7; full conditionals eqs 32-40, Section 4.1).
 *
 * Model and prior constants as in lmvb.h (V genes, N subpopulations, M = N - 1, r_i, d_i, mu_i,
 * D_i).  Full conditionals:
 *   Lambda | ... ~ Wishart(n0 + V + 1, scale Lambda_L^-1),
 *     Lambda_L = L0^-1 + q0 (K - K0)(K - K0)^T + sum_i (beta_i - K)(beta_i - K)^T   (eqs 32-34)
 *   K | ... ~ N((q0 K0 + sum_i beta_i) / (q0 + V), ((q0 + V) Lambda)^-1)           (eq 35)
 *   rho | ... ~ Gamma(a0 + V/2, rate b0 + 1/2 sum_i (r_i - mu_i - D_i^T beta_i)^2)  (eqs 36, 37)
 *   beta_i | ... ~ N(P^-1 (Lambda K + rho (r_i - mu_i) D_i), P^-1), P = Lambda + rho D_i D_i^T
 *                                                                                    (eqs 38-40)
 * The chain starts from the means of the priors (Lambda_1 = n0 L0, K_1 = K0, rho_0 = a0 / b0) and
 * iteration t draws every beta_i from (Lambda_t, K_t, rho_{t-1}), then rho_t, Lambda_{t+1} and
 * K_{t+1}.  Row t of the chain (t = 1, 2, ...) is (rho_t, K_t, Lambda_t).
 *
 * Draws.  Normal vectors as mean + C u, C the Cholesky factor of the covariance; rho and the
 * chi-square variates by the Marsaglia-Tsang sampler; Lambda by Bartlett's decomposition.  Random
 * numbers are counter-based (Philox4x32-10, key (seed mod 2^32, 0x47494253)): gene i of iteration t
 * takes block j (its normals 2j and 2j + 1) at counter (i mod 2^32, i div 2^32, t, j); the global
 * draws of iteration t take stream s at counter (k, 0, t, 0x80000000 + s) (s = 1 rho, 2 K, 3 the
 * below-diagonal normals of Bartlett's factor, 16 + j its diagonal j); a block gives two uniforms
 * (m + 1/2) 2^-53 and two Box-Muller normals.  The draws are thus a function of (seed, data,
 * prior) only: bitwise reproducible run to run, independent of the launch shape.
 *
 * Conventions (as in cavi.h; the status codes and cavi_last_error() are shared):
 *   - r (V) and d (V x N, row-major) are FP64 in DEVICE memory, caller-owned, 8-byte aligned,
 *     unchanged and alive until the handle is destroyed.  The library never copies or frees them.
 *   - Host arrays are FP64 and caller-owned; matrices are M x M row-major.
 *   - Work runs on the stream given at creation (hipStream_t as void*; NULL: a blocking stream of
 *     the handle's own).  Functions returning results to the host synchronise it.  A handle is not
 *     thread-safe.  The library allocates its own device memory: O(V / 256) doubles and the last
 *     65536 rows of the chain.
 *   - Limits: 1 <= V < 2^40, 2 <= N <= 8, n0 + V >= N - 1 and a0 + V/2 >= 1 (every Gamma draw has
 *     shape >= 1), at most 2^32 - 2 iterations.
 */
#ifndef GIBBS_H
#define GIBBS_H

#include <stddef.h>
#include <stdint.h>

#include "cavi.h"
#include "lmvb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gibbs_ctx gibbs_ctx;

/* Create a chain over r_dev (V) and d_dev (V x N) at its start.  prior NULL: the paper's constants
 * (as lmvb_create).  CAVI_E_INVAL: bad shape, NULL or misaligned pointer, invalid constants. */
cavi_status gibbs_create(gibbs_ctx **out, const double *r_dev, const double *d_dev, int64_t V, int32_t N,
                         const lmvb_prior *prior, uint64_t seed, void *hip_stream);

/* n >= 1 iterations.  Synchronises.  CAVI_E_NUMERIC if an iteration produced a non-finite value
 * or a matrix that is not positive definite (the chain keeps its last valid iteration). */
cavi_status gibbs_iterate(gibbs_ctx *h, int32_t n);

/* Rows first + 1 .. first + count of the chain (0-based first), each of the last 65536 rows:
 * rho (count), K (count x M), Lambda (count x M x M); any output may be NULL.  CAVI_E_INVAL for
 * rows not drawn yet or no longer kept. */
cavi_status gibbs_get_chain(gibbs_ctx *h, int64_t first, int32_t count, double *rho, double *K, double *Lam);

/* The chain's state after t iterations: t, rho_t, K_{t+1}, Lambda_{t+1} (the values the next
 * iteration draws from).  Any pointer may be NULL. */
cavi_status gibbs_get_state(gibbs_ctx *h, int64_t *t, double *rho, double *K, double *Lam);

/* The beta_i of the last iteration into DEVICE memory (V x M), recomputed from its counters.
 * CAVI_E_STATE before the first iteration. */
cavi_status gibbs_get_genes(gibbs_ctx *h, double *beta_dev);

/* Average duration (ms, HIP events on the handle's stream) of reps launches of the per-gene pass
 * of the next iteration (the chain is unchanged).  Synchronises. */
cavi_status gibbs_profile_pass(gibbs_ctx *h, int32_t reps, float *ms);

/* Release the handle (NULL is a no-op). */
cavi_status gibbs_destroy(gibbs_ctx *h);

#ifdef __cplusplus
}
#endif

#endif /* GIBBS_H */
