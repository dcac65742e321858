/*
 * FP64 CPU oracle for the mean-field (CAVI) sweep of the finite Gaussian
 * mixture that the GPU library implements.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code with the GPU path: nothing here is included by, or includes, anything
 * under the package's csrc/ or include/.
 *
 * Written from the paper's variational method (Section 3.4): the mean-field
 * factorisation (eqs 9 and 13), the lower bound (eqs 10-11) and the
 * coordinate update (eq 12), applied to the mixture
 *
 *   pi ~ Dir(alpha0 1_K);  tau_kg ~ Gamma(a0, rate b0);
 *   mu_kg | tau_kg ~ N(m0_g, 1/(beta0 tau_kg));
 *   z_n ~ Cat(pi);  x_ng | z_n = k ~ N(mu_kg, 1/tau_kg),
 *
 * with q = prod_n Cat(z_n | r_n) Dir(pi | alpha) prod_kg NG(mu,tau | m,beta,a,b).
 * The conjugate update forms follow eq 16 (shape = prior shape + half the
 * count), eq 17 (rate = prior rate + half a residual sum) and eq 24 (prior-
 * weighted mean); expectations follow eqs 26-31 (E[tau] = a/b as in eq 29).
 * Gamma is shape/rate ("inverse scale") as in eq 5.
 *
 * Steps (one sweep):
 *   S1  E ln pi_k = psi(alpha_k) - psi(sum alpha);  tbar = a/b;  E ln tau = psi(a) - ln b
 *   S2  l_nk = E ln pi_k + sum_g 1/2 [E ln tau - ln 2pi - tbar (x - m)^2 - 1/beta]
 *   S3  L_n = logsumexp_k l_nk;  r_nk = exp(l_nk - L_n);  H = -sum r (l - L)
 *   S4  N_k = sum_n r;  xbar = sum_n r x / N_k;  C = sum_n r (x - xbar)^2   (two passes)
 *   S5  alpha = alpha0 + N_k;  beta = beta0 + N_k;  m = (beta0 m0 + N_k xbar)/beta;
 *       a = a0 + N_k/2;  b = b0 + 1/2 [C + beta0 N_k (xbar - m0)^2 / beta]
 *   S6  lower bound at the updated q(pi), q(mu,tau) with the S3 responsibilities
 *   S7  converged when t >= 2 and |L_t - L_{t-1}| <= tol |L_t|
 * Standard initialisation (S0): k-means++ (D^2 sampling) seeds, with the
 * D^2 weights quantised to integers so that the draw is exact, then a hard
 * nearest-seed assignment followed by S5.
 *
 * Everything is plain loops in FP64 with no blocking or reordering; compile
 * with -ffp-contract=off.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OC_LN2PI 1.8378770664093454835606594728112
#define OC_PI 3.14159265358979323846264338327950

/* ------------------------------------------------------------------ special functions */

/* Digamma for x > 0: shift with psi(x) = psi(x+1) - 1/x until x >= 10, then
 * the asymptotic series psi(x) ~ ln x - 1/(2x) - sum_k B_2k / (2k x^2k)
 * (Abramowitz & Stegun 6.3.5 and 6.3.18), Bernoulli numbers B_2 .. B_14. */
double oc_digamma(double x)
{
    double acc = 0.0;
    while (x < 10.0) {
        acc -= 1.0 / x;
        x += 1.0;
    }
    double f = 1.0 / (x * x);
    double series = f * (1.0 / 12.0 - f * (1.0 / 120.0 - f * (1.0 / 252.0 - f * (1.0 / 240.0
                    - f * (1.0 / 132.0 - f * (691.0 / 32760.0 - f * (1.0 / 12.0)))))));
    return acc + log(x) - 0.5 / x - series;
}

double oc_lgamma(double x) { return lgamma(x); }

/* ------------------------------------------------------------------ SplitMix64 */

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014). */
uint64_t oc_splitmix64_next(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* floor(u53 * n / 2^53) with u53 the top 53 bits of one draw. */
static uint64_t scaled_draw(uint64_t *s, uint64_t n)
{
    uint64_t u = oc_splitmix64_next(s) >> 11;
    return (uint64_t)(((unsigned __int128)u * (unsigned __int128)n) >> 53);
}

/* ------------------------------------------------------------------ S1 */

void oc_expectations(int K, int G, const double *alpha, const double *a, const double *b,
                     double *elnpi, double *tbar, double *elntau)
{
    double asum = 0.0;
    for (int k = 0; k < K; ++k) asum += alpha[k];
    double psum = oc_digamma(asum);
    for (int k = 0; k < K; ++k) elnpi[k] = oc_digamma(alpha[k]) - psum;
    for (int i = 0; i < K * G; ++i) {
        tbar[i] = a[i] / b[i];
        elntau[i] = oc_digamma(a[i]) - log(b[i]);
    }
}

/* ------------------------------------------------------------------ S2 + S3 */

/* Responsibilities r[N*K] (row-major), optional log normalisers Ln[N];
 * returns the entropy H = -sum r ln r. */
double oc_estep(const float *X, int64_t N, int G, int K,
                const double *alpha, const double *m, const double *beta,
                const double *a, const double *b, double *r, double *Ln)
{
    double *elnpi = malloc(sizeof(double) * K);
    double *tbar = malloc(sizeof(double) * K * G);
    double *elntau = malloc(sizeof(double) * K * G);
    double *l = malloc(sizeof(double) * K);
    oc_expectations(K, G, alpha, a, b, elnpi, tbar, elntau);
    double H = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        const float *x = X + n * G;
        for (int k = 0; k < K; ++k) {
            double s = elnpi[k];
            for (int g = 0; g < G; ++g) {
                int i = k * G + g;
                double d = (double)x[g] - m[i];
                s += 0.5 * (elntau[i] - OC_LN2PI - tbar[i] * d * d - 1.0 / beta[i]);
            }
            l[k] = s;
        }
        double mx = l[0];
        for (int k = 1; k < K; ++k)
            if (l[k] > mx) mx = l[k];
        double se = 0.0;
        for (int k = 0; k < K; ++k) se += exp(l[k] - mx);
        double L = mx + log(se);
        for (int k = 0; k < K; ++k) {
            double rk = exp(l[k] - L);
            r[n * K + k] = rk;
            H -= rk * (l[k] - L);
        }
        if (Ln) Ln[n] = L;
    }
    free(elnpi);
    free(tbar);
    free(elntau);
    free(l);
    return H;
}

/* ------------------------------------------------------------------ S4 */

/* Nk[K], xbar[K*G], C[K*G] by two passes over the rows. */
void oc_stats(const float *X, int64_t N, int G, int K, const double *r,
              double *Nk, double *xbar, double *C)
{
    for (int k = 0; k < K; ++k) {
        Nk[k] = 0.0;
        for (int g = 0; g < G; ++g) {
            xbar[k * G + g] = 0.0;
            C[k * G + g] = 0.0;
        }
    }
    for (int64_t n = 0; n < N; ++n)
        for (int k = 0; k < K; ++k) {
            double rk = r[n * K + k];
            Nk[k] += rk;
            for (int g = 0; g < G; ++g) xbar[k * G + g] += rk * (double)X[n * G + g];
        }
    for (int k = 0; k < K; ++k)
        for (int g = 0; g < G; ++g)
            xbar[k * G + g] = Nk[k] > 0.0 ? xbar[k * G + g] / Nk[k] : 0.0;
    for (int64_t n = 0; n < N; ++n)
        for (int k = 0; k < K; ++k) {
            double rk = r[n * K + k];
            for (int g = 0; g < G; ++g) {
                double d = (double)X[n * G + g] - xbar[k * G + g];
                C[k * G + g] += rk * d * d;
            }
        }
}

/* ------------------------------------------------------------------ S5 */

/* prior = {alpha0, beta0, a0, b0}; m0[G]. */
void oc_update(int G, int K, const double *prior, const double *m0,
               const double *Nk, const double *xbar, const double *C,
               double *alpha, double *m, double *beta, double *a, double *b)
{
    double alpha0 = prior[0], beta0 = prior[1], a0 = prior[2], b0 = prior[3];
    for (int k = 0; k < K; ++k) {
        alpha[k] = alpha0 + Nk[k];
        for (int g = 0; g < G; ++g) {
            int i = k * G + g;
            double bt = beta0 + Nk[k];
            beta[i] = bt;
            m[i] = (beta0 * m0[g] + Nk[k] * xbar[i]) / bt;
            a[i] = a0 + 0.5 * Nk[k];
            double dm = xbar[i] - m0[g];
            b[i] = b0 + 0.5 * (C[i] + beta0 * Nk[k] * dm * dm / bt);
        }
    }
}

/* ------------------------------------------------------------------ S6 */

/* Lower bound from the statistics (Nk, xbar, C) of the responsibilities, the
 * entropy H of q(z) and the (updated) global factors. */
double oc_elbo(int G, int K, const double *prior, const double *m0,
               const double *Nk, const double *xbar, const double *C, double H,
               const double *alpha, const double *m, const double *beta,
               const double *a, const double *b)
{
    double alpha0 = prior[0], beta0 = prior[1], a0 = prior[2], b0 = prior[3];
    double *elnpi = malloc(sizeof(double) * K);
    double *tbar = malloc(sizeof(double) * K * G);
    double *elntau = malloc(sizeof(double) * K * G);
    oc_expectations(K, G, alpha, a, b, elnpi, tbar, elntau);

    double L = 0.0;
    /* E[ln p(X | Z, mu, tau)] */
    for (int k = 0; k < K; ++k)
        for (int g = 0; g < G; ++g) {
            int i = k * G + g;
            double dm = xbar[i] - m[i];
            L += 0.5 * (Nk[k] * (elntau[i] - OC_LN2PI) - tbar[i] * (C[i] + Nk[k] * dm * dm)
                        - Nk[k] / beta[i]);
        }
    /* E[ln p(Z | pi)] */
    for (int k = 0; k < K; ++k) L += Nk[k] * elnpi[k];
    /* E[ln p(pi)] - E[ln q(pi)] */
    double asum = 0.0;
    for (int k = 0; k < K; ++k) asum += alpha[k];
    L += lgamma(K * alpha0) - K * lgamma(alpha0);
    for (int k = 0; k < K; ++k) L += (alpha0 - 1.0) * elnpi[k];
    L -= lgamma(asum);
    for (int k = 0; k < K; ++k) L -= -lgamma(alpha[k]) + (alpha[k] - 1.0) * elnpi[k];
    /* E[ln p(mu, tau)] - E[ln q(mu, tau)] */
    for (int i = 0; i < K * G; ++i) {
        int g = i % G;
        double dm0 = m[i] - m0[g];
        L += 0.5 * log(beta0 / (2.0 * OC_PI)) + 0.5 * elntau[i]
             - 0.5 * beta0 * (tbar[i] * dm0 * dm0 + 1.0 / beta[i])
             + a0 * log(b0) - lgamma(a0) + (a0 - 1.0) * elntau[i] - b0 * tbar[i];
        L -= 0.5 * log(beta[i] / (2.0 * OC_PI)) + 0.5 * elntau[i] - 0.5
             + a[i] * log(b[i]) - lgamma(a[i]) + (a[i] - 1.0) * elntau[i] - a[i];
    }
    /* -E[ln q(Z)] */
    L += H;
    free(elnpi);
    free(tbar);
    free(elntau);
    return L;
}

/* The same bound evaluated term by term per observation from r (an
 * independent second evaluation used by the tests). */
double oc_elbo_direct(const float *X, int64_t N, int G, int K, const double *prior,
                      const double *m0, const double *r,
                      const double *alpha, const double *m, const double *beta,
                      const double *a, const double *b)
{
    double alpha0 = prior[0], beta0 = prior[1], a0 = prior[2], b0 = prior[3];
    double *elnpi = malloc(sizeof(double) * K);
    double *tbar = malloc(sizeof(double) * K * G);
    double *elntau = malloc(sizeof(double) * K * G);
    oc_expectations(K, G, alpha, a, b, elnpi, tbar, elntau);
    double L = 0.0;
    for (int64_t n = 0; n < N; ++n)
        for (int k = 0; k < K; ++k) {
            double rk = r[n * K + k];
            double t = elnpi[k];
            for (int g = 0; g < G; ++g) {
                int i = k * G + g;
                double d = (double)X[n * G + g] - m[i];
                t += 0.5 * (elntau[i] - OC_LN2PI - tbar[i] * d * d - 1.0 / beta[i]);
            }
            L += rk * t;
            if (rk > 0.0) L -= rk * log(rk);
        }
    /* Dirichlet terms via the KL divergence of two Dirichlets */
    double asum = 0.0;
    for (int k = 0; k < K; ++k) asum += alpha[k];
    double kl_pi = lgamma(asum) - lgamma(K * alpha0);
    for (int k = 0; k < K; ++k)
        kl_pi += -lgamma(alpha[k]) + lgamma(alpha0) + (alpha[k] - alpha0) * elnpi[k];
    L -= kl_pi;
    /* Normal-Gamma terms via KL(q || p) = KL_Gamma + E_q[tau] KL_Normal part */
    for (int i = 0; i < K * G; ++i) {
        int g = i % G;
        double kl_g = (a[i] - a0) * oc_digamma(a[i]) - lgamma(a[i]) + lgamma(a0)
                      + a0 * (log(b[i]) - log(b0)) + a[i] * (b0 - b[i]) / b[i];
        double dm = m[i] - m0[g];
        double kl_n = 0.5 * (beta0 / beta[i] - 1.0 - log(beta0 / beta[i]))
                      + 0.5 * beta0 * tbar[i] * dm * dm;
        L -= kl_g + kl_n;
    }
    free(elnpi);
    free(tbar);
    free(elntau);
    return L;
}

/* ------------------------------------------------------------------ one sweep */

/* S1..S6 in place on the state; returns the bound.  r_out (N*K) optional. */
double oc_sweep(const float *X, int64_t N, int G, int K, const double *prior, const double *m0,
                double *alpha, double *m, double *beta, double *a, double *b, double *r_out)
{
    double *r = r_out ? r_out : malloc(sizeof(double) * N * K);
    double *Nk = malloc(sizeof(double) * K);
    double *xbar = malloc(sizeof(double) * K * G);
    double *C = malloc(sizeof(double) * K * G);
    double H = oc_estep(X, N, G, K, alpha, m, beta, a, b, r, NULL);
    oc_stats(X, N, G, K, r, Nk, xbar, C);
    oc_update(G, K, prior, m0, Nk, xbar, C, alpha, m, beta, a, b);
    double L = oc_elbo(G, K, prior, m0, Nk, xbar, C, H, alpha, m, beta, a, b);
    if (!r_out) free(r);
    free(Nk);
    free(xbar);
    free(C);
    return L;
}

/* The same sweep with the rows split over nthreads contiguous ranges (OpenMP):
 * each thread forms the S2-S3 responsibilities and entropy of its rows and the
 * S4 sums over them (first N_k and sum r x, then, after xbar, sum r (x-xbar)^2),
 * and the per-thread FP64 sums are added in thread order.  With one thread
 * every sum is taken in row order, as in oc_sweep.  Used to time the oracle on
 * all host cores and to run it at full workload sizes; the arithmetic per row
 * is that of oc_estep and oc_stats.  Returns the bound; *used receives the
 * number of threads that ran (optional). */
double oc_sweep_mt(const float *X, int64_t N, int G, int K, const double *prior, const double *m0,
                   double *alpha, double *m, double *beta, double *a, double *b, int nthreads, int *used)
{
    if (nthreads < 1) nthreads = 1;
    const size_t KG = (size_t)K * G;
    double *elnpi = malloc(sizeof(double) * K);
    double *tbar = malloc(sizeof(double) * KG);
    double *elntau = malloc(sizeof(double) * KG);
    double *r = malloc(sizeof(double) * (size_t)N * K);
    double *Ht = calloc((size_t)nthreads, sizeof(double));
    double *Nkt = calloc((size_t)nthreads * K, sizeof(double));
    double *St = calloc((size_t)nthreads * KG, sizeof(double));
    double *Ct = calloc((size_t)nthreads * KG, sizeof(double));
    double *Nk = calloc((size_t)K, sizeof(double));
    double *xbar = calloc(KG, sizeof(double));
    double *C = calloc(KG, sizeof(double));
    int nt_used = 1;
    oc_expectations(K, G, alpha, a, b, elnpi, tbar, elntau);
#pragma omp parallel num_threads(nthreads)
    {
        const int t = omp_get_thread_num(), nt = omp_get_num_threads();
        const int64_t lo = N * t / nt, hi = N * (t + 1) / nt;
        double *l = malloc(sizeof(double) * K);
        double H = 0.0;
        for (int64_t n = lo; n < hi; ++n) {
            const float *x = X + n * G;
            for (int k = 0; k < K; ++k) {
                double s = elnpi[k];
                for (int g = 0; g < G; ++g) {
                    int i = k * G + g;
                    double d = (double)x[g] - m[i];
                    s += 0.5 * (elntau[i] - OC_LN2PI - tbar[i] * d * d - 1.0 / beta[i]);
                }
                l[k] = s;
            }
            double mx = l[0];
            for (int k = 1; k < K; ++k)
                if (l[k] > mx) mx = l[k];
            double se = 0.0;
            for (int k = 0; k < K; ++k) se += exp(l[k] - mx);
            double L = mx + log(se);
            for (int k = 0; k < K; ++k) {
                double rk = exp(l[k] - L);
                r[n * K + k] = rk;
                H -= rk * (l[k] - L);
            }
        }
        Ht[t] = H;
        double *nk = Nkt + (size_t)t * K, *sx = St + (size_t)t * KG, *cc = Ct + (size_t)t * KG;
        for (int64_t n = lo; n < hi; ++n)
            for (int k = 0; k < K; ++k) {
                double rk = r[n * K + k];
                nk[k] += rk;
                for (int g = 0; g < G; ++g) sx[k * G + g] += rk * (double)X[n * G + g];
            }
#pragma omp barrier
#pragma omp single
        {
            nt_used = nt;
            for (int u = 0; u < nt; ++u)
                for (int k = 0; k < K; ++k) Nk[k] += Nkt[(size_t)u * K + k];
            for (int u = 0; u < nt; ++u)
                for (size_t i = 0; i < KG; ++i) xbar[i] += St[(size_t)u * KG + i];
            for (int k = 0; k < K; ++k)
                for (int g = 0; g < G; ++g)
                    xbar[k * G + g] = Nk[k] > 0.0 ? xbar[k * G + g] / Nk[k] : 0.0;
        }
        for (int64_t n = lo; n < hi; ++n)
            for (int k = 0; k < K; ++k) {
                double rk = r[n * K + k];
                for (int g = 0; g < G; ++g) {
                    double d = (double)X[n * G + g] - xbar[k * G + g];
                    cc[k * G + g] += rk * d * d;
                }
            }
        free(l);
    }
    double H = 0.0;
    for (int u = 0; u < nt_used; ++u) H += Ht[u];
    for (int u = 0; u < nt_used; ++u)
        for (size_t i = 0; i < KG; ++i) C[i] += Ct[(size_t)u * KG + i];
    oc_update(G, K, prior, m0, Nk, xbar, C, alpha, m, beta, a, b);
    double Lb = oc_elbo(G, K, prior, m0, Nk, xbar, C, H, alpha, m, beta, a, b);
    if (used) *used = nt_used;
    free(elnpi);
    free(tbar);
    free(elntau);
    free(r);
    free(Ht);
    free(Nkt);
    free(St);
    free(Ct);
    free(Nk);
    free(xbar);
    free(C);
    return Lb;
}

/* S7: sweeps until converged or max_sweeps.  elbo_trace[max_sweeps] optional.
 * Returns the number of sweeps run; *converged set to 0/1. */
int oc_run(const float *X, int64_t N, int G, int K, const double *prior, const double *m0,
           double *alpha, double *m, double *beta, double *a, double *b,
           int max_sweeps, double tol, double *elbo_trace, int *converged)
{
    double prev = 0.0;
    *converged = 0;
    for (int t = 1; t <= max_sweeps; ++t) {
        double L = oc_sweep(X, N, G, K, prior, m0, alpha, m, beta, a, b, NULL);
        if (elbo_trace) elbo_trace[t - 1] = L;
        if (t >= 2 && fabs(L - prev) <= tol * fabs(L)) {
            *converged = 1;
            return t;
        }
        prev = L;
    }
    return max_sweeps;
}

/* ------------------------------------------------------------------ S0 */

static double sqdist(const float *X, int G, int64_t i, int64_t j)
{
    double s = 0.0;
    for (int g = 0; g < G; ++g) {
        double d = (double)X[i * G + g] - (double)X[j * G + g];
        s += d * d;
    }
    return s;
}

/* k-means++ seed rows (seeds[K]) from SplitMix64(seed).  The D^2 weights are
 * w_n = floor(minD2_n * 2^e) with the largest e that keeps sum_n w_n < 2^62,
 * so the draw "smallest n with cumsum(w)_n > t", t = floor(u * W), is exact. */
void oc_kmeanspp_seeds(const float *X, int64_t N, int G, int K, uint64_t seed, int64_t *seeds)
{
    uint64_t s = seed;
    double *mind = malloc(sizeof(double) * N);
    seeds[0] = (int64_t)scaled_draw(&s, (uint64_t)N);
    for (int64_t n = 0; n < N; ++n) mind[n] = sqdist(X, G, n, seeds[0]);
    int clog2n = 0;
    while (((int64_t)1 << clog2n) < N) ++clog2n;
    for (int j = 1; j < K; ++j) {
        double mx = 0.0;
        for (int64_t n = 0; n < N; ++n)
            if (mind[n] > mx) mx = mind[n];
        if (mx == 0.0) {
            seeds[j] = (int64_t)scaled_draw(&s, (uint64_t)N);
        } else {
            int E;
            frexp(mx, &E);
            int e = 62 - E - clog2n;
            uint64_t W = 0;
            for (int64_t n = 0; n < N; ++n) W += (uint64_t)floor(ldexp(mind[n], e));
            uint64_t t = scaled_draw(&s, W);
            uint64_t cum = 0;
            int64_t pick = N - 1;
            for (int64_t n = 0; n < N; ++n) {
                cum += (uint64_t)floor(ldexp(mind[n], e));
                if (cum > t) {
                    pick = n;
                    break;
                }
            }
            seeds[j] = pick;
        }
        for (int64_t n = 0; n < N; ++n) {
            double d = sqdist(X, G, n, seeds[j]);
            if (d < mind[n]) mind[n] = d;
        }
    }
    free(mind);
}

/* Standard initial state: hard nearest-seed responsibilities (ties to the
 * lowest seed index), then S5.  r_out (N*K) optional. */
void oc_init_standard(const float *X, int64_t N, int G, int K, const double *prior,
                      const double *m0, uint64_t seed,
                      double *alpha, double *m, double *beta, double *a, double *b,
                      int64_t *seeds_out, double *r_out)
{
    int64_t *seeds = seeds_out ? seeds_out : malloc(sizeof(int64_t) * K);
    double *r = r_out ? r_out : malloc(sizeof(double) * N * K);
    double *Nk = malloc(sizeof(double) * K);
    double *xbar = malloc(sizeof(double) * K * G);
    double *C = malloc(sizeof(double) * K * G);
    oc_kmeanspp_seeds(X, N, G, K, seed, seeds);
    for (int64_t n = 0; n < N; ++n) {
        int best = 0;
        double bd = sqdist(X, G, n, seeds[0]);
        for (int j = 1; j < K; ++j) {
            double d = sqdist(X, G, n, seeds[j]);
            if (d < bd) {
                bd = d;
                best = j;
            }
        }
        for (int k = 0; k < K; ++k) r[n * K + k] = (k == best) ? 1.0 : 0.0;
    }
    oc_stats(X, N, G, K, r, Nk, xbar, C);
    oc_update(G, K, prior, m0, Nk, xbar, C, alpha, m, beta, a, b);
    if (!seeds_out) free(seeds);
    if (!r_out) free(r);
    free(Nk);
    free(xbar);
    free(C);
}
