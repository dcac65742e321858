// gfx950 kernels and C ABI (include/lmvb.h) of the variational Bayes for the paper's own
// linear-mixing model (Section 3.3, eqs 2-8), with the updates of eqs 16-31 in the order of the
// steps of Section 3.5.
//
// One sweep is three launches:
//   k_lm_pass<M>     one thread per gene: q(beta_i) from the current coefficients (eqs 20, 21),
//                    its moments (eqs 26, 27), and the gene's terms of the sums that the global
//                    updates need (sum m_i, sum E[beta_i beta_i^T], the bracket of eq 17 and
//                    ln|P_i|); FP64 sums per chunk of 256 ppt genes in a fixed order, with
//                    ppt = min(32, max(1, ceil(V / 2^18))) genes per thread (a function of V only:
//                    small problems spread over more workgroups);
//   k_lm_reduce      the chunk sums in 16 contiguous groups, each in chunk order;
//   k_lm_global<M>   the groups in order, then q(K, Lambda) (eqs 24, 25), the lower bound, the
//                    convergence test, and q(rho) (eqs 16, 17) with the coefficients E[rho],
//                    E[Lambda], E[Lambda K] (eqs 28, 29, 31) of the next pass.
// The gene factors are not stored: they are a function of the data and of the coefficients of the
// pass that formed them, which the state keeps (lmvb_get_genes recomputes them).
// Everything is FP64, as in the paper.  k_lm_pass and k_lm_reduce are shared with the EM
// (linmix.h).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/lmvb.h"
#include "cavi_impl.h"
#include "devmath.h"
#include "linmix.h"

namespace {

struct State {
    double a_rho, b_rho;   // q(rho)
    double K0K[kMaxM];     // q(K | Lambda) mean
    double W[kMaxM * kMaxM];  // q(Lambda) scale matrix
    double nu, kappa;
    double elbo, tol;
    int32_t sweeps, call_sweeps, max_call, stop_on_conv, converged, numeric, swept, pad;
    Coef coef;  // next pass
    Coef used;  // the pass that formed the current q(beta)
};

// The M-sized part of a coefficient block, element by element (a whole-struct copy is held in
// registers across the update and spills).
template <int M>
__device__ void copy_coef(Coef &dst, const Coef &src)
{
    dst.a_rho = src.a_rho;
    dst.b_rho = src.b_rho;
    dst.Erho = src.Erho;
    for (int i = 0; i < M * M; ++i) dst.ELam[i] = src.ELam[i];
    for (int i = 0; i < M; ++i) dst.ELamK[i] = src.ELamK[i];
}

// Coefficients of the next pass from q(rho) = Gamma(a, b) and q(K, Lambda) (eqs 28, 29, 31).
template <int M>
__device__ void next_coef(Coef &c, double a, double b, const double *W, const double *K0K, double nu)
{
    c.a_rho = a;
    c.b_rho = b;
    c.Erho = a / b;
    for (int i = 0; i < M; ++i) {
        double t = 0.0;
        for (int j = 0; j < M; ++j) {
            c.ELam[i * M + j] = nu * W[i * M + j];
            t += W[i * M + j] * K0K[j];
        }
        c.ELamK[i] = nu * t;
    }
}

// One workgroup of three waves, each on its own SIMD, so that independent work overlaps:
//   wave 0: lanes s < S add up sum s over the 16 groups in order; lane 0 gathers them and forms
//           q(K, Lambda) (eqs 24, 25) and the parts of the bound that need no special function;
//   wave 1: digamma of (nu + 1 - j) / 2 on lanes j - 1 < M (Wishart expectations) and of a_rho on
//           lane M;
//   wave 2: lgamma of the same arguments.
// Then wave 0's lane 0 finishes the bound, the convergence test and q(rho).
template <int M>
__global__ __launch_bounds__(192) void k_lm_global(Shape sh, State *st, const Prior *pr, int init_mode,
                                                   const double *__restrict__ level1, double *__restrict__ hist)
{
    if (!init_mode && skipped(st)) return;
    constexpr int S = M + M * (M + 1) / 2 + 2;
    static_assert(S <= 64, "one wave for the sums");
    __shared__ double sp[2][kMaxM + 2];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double V = (double)sh.V;
    const double nu = pr->n0 + V, kappa = pr->q0 + V;
    // q(rho) of this sweep's pass (the coefficient block itself is copied to st->used at the end)
    const double used_a = st->coef.a_rho, used_b = st->coef.b_rho;
    double tot[S];
    double K0K[M], W[M * M], Ebb[M * M], lndetW = 0.0, trWA = 0.0, trL0W = 0.0, dKWdK = 0.0;
    bool bad = false;
    if (wv == 0) {
        double v = 0.0;
        if (lane < S) {
            v = level1[lane];
            for (int b = 1; b < kGroups; ++b) v += level1[(size_t)b * kMaxS + lane];
        }
#pragma unroll
        for (int q = 0; q < S; ++q) tot[q] = __shfl(v, q, 64);
        if (lane == 0 && !init_mode) {
            // q(K, Lambda): eqs 24 and 25 with the new q(beta)
            double Winv[M * M];
            for (int i = 0; i < M; ++i) K0K[i] = (tot[i] + pr->q0 * pr->K0[i]) / (V + pr->q0);
            for (int i = 0; i < M; ++i)
                for (int k = i; k < M; ++k) {
                    Ebb[i * M + k] = tot[tri(M, i, k)];
                    Ebb[k * M + i] = tot[tri(M, i, k)];
                }
            for (int i = 0; i < M; ++i)
                for (int k = 0; k < M; ++k)
                    Winv[i * M + k] = pr->L0inv[i * M + k] + Ebb[i * M + k] + pr->q0 * pr->K0[i] * pr->K0[k]
                                      - (pr->q0 + V) * K0K[i] * K0K[k];
            double lndetWinv = 0.0;
            bad = !spd_inverse<M>(Winv, W, lndetWinv);
            lndetW = -lndetWinv;
            for (int i = 0; i < M; ++i)
                for (int k = 0; k < M; ++k) {
                    const double A = Ebb[k * M + i] - tot[k] * K0K[i] - K0K[k] * tot[i] + V * K0K[k] * K0K[i];
                    trWA += W[i * M + k] * A;
                    trL0W += pr->L0inv[i * M + k] * W[k * M + i];
                    dKWdK += (K0K[i] - pr->K0[i]) * W[i * M + k] * (K0K[k] - pr->K0[k]);
                }
        }
    } else if (!init_mode && lane <= M) {
        const double x = lane < M ? 0.5 * (nu - lane) : used_a;  // (nu + 1 - j) / 2 for j = lane + 1
        if (wv == 1)
            sp[0][lane] = cavi::dev_digamma(x);
        else
            sp[1][lane] = cavi::dev_lgamma(x);
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double rho_stat = tot[S - 2];
    if (init_mode) {
        // initial state (Section 3.5) and the coefficients of the first pass
        st->a_rho = pr->a0;
        st->b_rho = pr->b0;
        double K0[M], W0[M * M];
        for (int i = 0; i < M; ++i) K0[i] = 1.0 / (M + 1);
        for (int i = 0; i < M * M; ++i) W0[i] = pr->L0inv[i];
        for (int i = 0; i < M; ++i) st->K0K[i] = K0[i];
        for (int i = 0; i < M * M; ++i) st->W[i] = W0[i];
        st->nu = nu;
        st->kappa = kappa;
        st->elbo = 0.0;
        st->sweeps = 0;
        st->call_sweeps = 0;
        st->converged = 0;
        st->swept = 0;
        const double a1 = pr->a0 + 0.5 * V, b1 = pr->b0 + 0.5 * rho_stat;
        st->numeric = isfinite(b1) ? 0 : 1;
        next_coef<M>(st->coef, a1, b1, W0, K0, nu);
        return;
    }
    // the lower bound at q(rho) of this sweep, the new q(beta) and the new q(K, Lambda)
    const double a = used_a, b = used_b;
    const double Erho = a / b, Elnrho = sp[0][M] - log(b);
    double sdig = 0.0, slg = 0.0;
    for (int j = 0; j < M; ++j) {
        sdig += sp[0][j];
        slg += sp[1][j];
    }
    const double ElndetL = sdig + M * kLn2 + lndetW;
    const double t_lik = 0.5 * V * Elnrho - 0.5 * V * kLn2Pi - 0.5 * Erho * rho_stat;
    const double t_beta = 0.5 * V * ElndetL - 0.5 * V * M * kLn2Pi - 0.5 * (nu * trWA + V * M / kappa);
    const double t_rho = pr->a0 * log(pr->b0) - pr->lg_a0 + (pr->a0 - 1.0) * Elnrho - pr->b0 * Erho;
    const double t_K = 0.5 * M * log(pr->q0 / (2.0 * M_PI)) + 0.5 * ElndetL - 0.5 * pr->q0 * (nu * dKWdK + M / kappa);
    const double t_L = 0.5 * (pr->n0 - M - 1.0) * ElndetL - 0.5 * nu * trL0W + pr->lnB0;
    const double h_rho = a - log(b) + sp[1][M] + (1.0 - a) * sp[0][M];
    const double h_beta = 0.5 * V * M * (1.0 + kLn2Pi) - 0.5 * tot[S - 1];
    const double h_K = -(0.5 * M * log(kappa / (2.0 * M_PI)) + 0.5 * ElndetL - 0.5 * M);
    const double lnBW = -0.5 * nu * lndetW - 0.5 * nu * M * kLn2 - 0.25 * M * (M - 1) * kLnPi - slg;
    const double h_L = -lnBW - 0.5 * (nu - M - 1.0) * ElndetL + 0.5 * nu * M;
    const double L = t_lik + t_beta + t_rho + t_K + t_L + h_rho + h_beta + h_K + h_L;
    // q(rho) for the next sweep from the new q(beta) (eqs 16, 17)
    const double a1 = pr->a0 + 0.5 * V, b1 = pr->b0 + 0.5 * rho_stat;
    bad = bad || !isfinite(L) || !isfinite(b1) || !(b1 > 0.0);
    for (int i = 0; i < M; ++i) bad = bad || !isfinite(K0K[i]);
    if (bad) {
        st->numeric = 1;
        return;
    }
    const int t = st->call_sweeps + 1;
    if (t >= 2 && fabs(L - st->elbo) <= st->tol * fabs(L)) st->converged = 1;
    hist[(t - 1) % kHistCap] = L;
    st->elbo = L;
    st->call_sweeps = t;
    st->sweeps += 1;
    st->a_rho = a;
    st->b_rho = b;
    for (int i = 0; i < M; ++i) st->K0K[i] = K0K[i];
    for (int i = 0; i < M * M; ++i) st->W[i] = W[i];
    st->nu = nu;
    st->kappa = kappa;
    copy_coef<M>(st->used, st->coef);
    st->swept = 1;
    next_coef<M>(st->coef, a1, b1, W, K0K, nu);
}

// The gene factors of the current state: from the coefficients of the pass that formed them, or
// the initial values (m_i = 1/N, P_i = L0) before the first sweep.
template <int M>
__global__ __launch_bounds__(kThreads) void k_lm_genes(Shape sh, const double *__restrict__ r,
                                                        const double *__restrict__ d, const State *st,
                                                        const Prior *pr, double *m_out, double *P_out)
{
    constexpr int N = M + 1;
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g >= sh.V) return;
    double m[M], P[M][M];
    if (!st->swept) {
        for (int i = 0; i < M; ++i) {
            m[i] = 1.0 / N;
            for (int k = 0; k < M; ++k) P[i][k] = pr->L0[i * M + k];
        }
    } else {
        const Coef &c = st->used;
        double dv[N], D[M], Sg[M][M], detP;
#pragma unroll
        for (int q = 0; q < N; ++q) dv[q] = d[g * N + q];
#pragma unroll
        for (int q = 0; q < M; ++q) D[q] = dv[q] - dv[N - 1];
        gene_factor<M>(D, r[g] - dv[N - 1], c, m, Sg, detP);
        for (int i = 0; i < M; ++i)
            for (int k = 0; k < M; ++k) P[i][k] = c.ELam[i * M + k] + c.Erho * D[i] * D[k];
    }
    if (m_out)
        for (int i = 0; i < M; ++i) m_out[g * M + i] = m[i];
    if (P_out)
        for (int i = 0; i < M; ++i)
            for (int k = 0; k < M; ++k) P_out[(g * M + i) * M + k] = P[i][k];
}

__global__ void k_lm_ctl(State *st, int max_call, int stop_on_conv, double tol)
{
    st->max_call = max_call;
    st->stop_on_conv = stop_on_conv;
    st->tol = tol;
    st->call_sweeps = 0;
    st->converged = 0;
    st->numeric = 0;
}


template <int M>
hipError_t launch_sweep(const Shape &sh, const double *r, const double *d, State *st, const Prior *pr,
                        double *partials, double *level1, double *hist, hipStream_t s)
{
    hipLaunchKernelGGL((k_lm_pass<M, false, State>), dim3(sh.nchunk), dim3(kThreads), 0, s, sh, r, d, st, pr, partials);
    launch_lm_reduce(sh, st, 0, partials, level1, s);
    hipLaunchKernelGGL((k_lm_global<M>), dim3(1), dim3(192), 0, s, sh, st, pr, 0, level1, hist);
    return hipGetLastError();
}

template <int M>
hipError_t launch_init(const Shape &sh, const double *r, const double *d, State *st, const Prior *pr,
                       double *partials, double *level1, double *hist, hipStream_t s)
{
    hipLaunchKernelGGL((k_lm_pass<M, true, State>), dim3(sh.nchunk), dim3(kThreads), 0, s, sh, r, d, st, pr, partials);
    launch_lm_reduce(sh, st, 1, partials, level1, s);
    hipLaunchKernelGGL((k_lm_global<M>), dim3(1), dim3(192), 0, s, sh, st, pr, 1, level1, hist);
    return hipGetLastError();
}

template <int M>
hipError_t launch_genes(const Shape &sh, const double *r, const double *d, const State *st, const Prior *pr,
                        double *m, double *P, hipStream_t s)
{
    const int64_t nb = (sh.V + kThreads - 1) / kThreads;
    hipLaunchKernelGGL((k_lm_genes<M>), dim3((unsigned)nb), dim3(kThreads), 0, s, sh, r, d, st, pr, m, P);
    return hipGetLastError();
}

hipError_t sweep_M(int M, const Shape &sh, const double *r, const double *d, State *st, const Prior *pr,
                   double *partials, double *level1, double *hist, hipStream_t s)
{
#define CALL(K) launch_sweep<K>(sh, r, d, st, pr, partials, level1, hist, s)
    switch (M) {
    case 1: return CALL(1);
    case 2: return CALL(2);
    case 3: return CALL(3);
    case 4: return CALL(4);
    case 5: return CALL(5);
    case 6: return CALL(6);
    default: return CALL(7);
    }
#undef CALL
}

template <int M>
hipError_t launch_pass(const Shape &sh, const double *r, const double *d, State *st, const Prior *pr,
                       double *partials, hipStream_t s)
{
    hipLaunchKernelGGL((k_lm_pass<M, false, State>), dim3(sh.nchunk), dim3(kThreads), 0, s, sh, r, d, st, pr, partials);
    return hipGetLastError();
}

hipError_t pass_M(int M, const Shape &sh, const double *r, const double *d, State *st, const Prior *pr,
                  double *partials, hipStream_t s)
{
#define CALL(K) launch_pass<K>(sh, r, d, st, pr, partials, s)
    switch (M) {
    case 1: return CALL(1);
    case 2: return CALL(2);
    case 3: return CALL(3);
    case 4: return CALL(4);
    case 5: return CALL(5);
    case 6: return CALL(6);
    default: return CALL(7);
    }
#undef CALL
}

hipError_t init_M(int M, const Shape &sh, const double *r, const double *d, State *st, const Prior *pr,
                  double *partials, double *level1, double *hist, hipStream_t s)
{
#define CALL(K) launch_init<K>(sh, r, d, st, pr, partials, level1, hist, s)
    switch (M) {
    case 1: return CALL(1);
    case 2: return CALL(2);
    case 3: return CALL(3);
    case 4: return CALL(4);
    case 5: return CALL(5);
    case 6: return CALL(6);
    default: return CALL(7);
    }
#undef CALL
}

hipError_t genes_M(int M, const Shape &sh, const double *r, const double *d, const State *st, const Prior *pr,
                   double *m, double *P, hipStream_t s)
{
#define CALL(K) launch_genes<K>(sh, r, d, st, pr, m, P, s)
    switch (M) {
    case 1: return CALL(1);
    case 2: return CALL(2);
    case 3: return CALL(3);
    case 4: return CALL(4);
    case 5: return CALL(5);
    case 6: return CALL(6);
    default: return CALL(7);
    }
#undef CALL
}

}  // namespace

struct lmvb_ctx {
    Shape sh{};
    const double *r = nullptr, *d = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    State *st = nullptr;   // device
    Prior *pr = nullptr;   // device
    double *partials = nullptr, *level1 = nullptr, *hist = nullptr;
    bool ready = false;
};

extern "C" {

cavi_status lmvb_create(lmvb_ctx **out, const double *r_dev, const double *d_dev, int64_t V, int32_t N,
                        const lmvb_prior *prior, void *hip_stream)
{
    if (!out) return lfail(CAVI_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!r_dev || !d_dev) return lfail(CAVI_E_INVAL, "r_dev or d_dev is NULL");
    if ((((uintptr_t)r_dev) & 7) || (((uintptr_t)d_dev) & 7)) return lfail(CAVI_E_INVAL, "r_dev or d_dev is not 8-byte aligned");
    if (V < 1 || V >= ((int64_t)1 << 40)) return lfail(CAVI_E_INVAL, "V=%lld outside [1, 2^40)", (long long)V);
    if (N < 2 || N > kMaxM + 1) return lfail(CAVI_E_INVAL, "N=%d outside [2, %d]", N, kMaxM + 1);
    const int M = N - 1;
    Prior p{};
    double lndetL0 = 0.0;
    if (const char *why = fill_prior(prior, M, p, &lndetL0)) return lfail(CAVI_E_INVAL, "%s", why);
    if (!(p.n0 + (double)V > M - 1)) return lfail(CAVI_E_INVAL, "n0 + V must exceed N - 2 (a proper posterior Wishart)");
    if (p.n0 > M - 1) {
        double s = 0.0;
        for (int j = 1; j <= M; ++j) s += lgamma(0.5 * (p.n0 + 1 - j));
        p.lnB0 = -0.5 * p.n0 * lndetL0 - 0.5 * p.n0 * M * kLn2 - 0.25 * M * (M - 1) * kLnPi - s;
    }
    p.lg_a0 = lgamma(p.a0);
    lmvb_ctx *h = new lmvb_ctx;
    h->sh = make_shape(V, N);
    h->r = r_dev;
    h->d = d_dev;
    hipError_t e = hipSuccess;
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreate(&h->stream);
        if (e != hipSuccess) {
            delete h;
            return lfail(CAVI_E_HIP, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        h->own_stream = true;
    }
    if ((e = hipMalloc(&h->st, sizeof(State))) != hipSuccess || (e = hipMalloc(&h->pr, sizeof(Prior))) != hipSuccess ||
        (e = hipMalloc(&h->partials, sizeof(double) * (size_t)h->sh.nchunk * h->sh.S)) != hipSuccess ||
        (e = hipMalloc(&h->level1, sizeof(double) * kGroups * kMaxS)) != hipSuccess ||
        (e = hipMalloc(&h->hist, sizeof(double) * kHistCap)) != hipSuccess) {
        (void)hipGetLastError();
        lmvb_destroy(h);
        return lfail(CAVI_E_NOMEM, "device allocation: %s", hipGetErrorString(e));
    }
    State s0{};
    e = hipMemcpyAsync(h->pr, &p, sizeof(Prior), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h->st, &s0, sizeof(State), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        lmvb_destroy(h);
        return lfail(CAVI_E_HIP, "upload: %s", hipGetErrorString(e));
    }
    *out = h;
    return CAVI_OK;
}

cavi_status lmvb_init(lmvb_ctx *h)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    LCHK(init_M(h->sh.M, h->sh, h->r, h->d, h->st, h->pr, h->partials, h->level1, h->hist, h->stream));
    State s;
    LCHK(hipMemcpyAsync(&s, h->st, sizeof(State), hipMemcpyDeviceToHost, h->stream));
    LCHK(hipStreamSynchronize(h->stream));
    if (s.numeric) return lfail(CAVI_E_NUMERIC, "the initial statistic of eq 17 is not finite");
    h->ready = true;
    return CAVI_OK;
}

static cavi_status enqueue(lmvb_ctx *h, int n, int max_call, int stop_on_conv, double tol, bool begin)
{
    if (begin) hipLaunchKernelGGL(k_lm_ctl, dim3(1), dim3(1), 0, h->stream, h->st, max_call, stop_on_conv, tol);
    for (int i = 0; i < n; ++i)
        LCHK(sweep_M(h->sh.M, h->sh, h->r, h->d, h->st, h->pr, h->partials, h->level1, h->hist, h->stream));
    return CAVI_OK;
}

cavi_status lmvb_sweep(lmvb_ctx *h, int32_t n, double *elbo_host)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    if (!h->ready) return lfail(CAVI_E_STATE, "lmvb_init has not run");
    if (n < 1 || n > kHistCap) return lfail(CAVI_E_INVAL, "n=%d outside [1, %d]", n, kHistCap);
    cavi_status st = enqueue(h, n, n, 0, 0.0, true);
    if (st != CAVI_OK) return st;
    State s;
    LCHK(hipMemcpyAsync(&s, h->st, sizeof(State), hipMemcpyDeviceToHost, h->stream));
    if (elbo_host) LCHK(hipMemcpyAsync(elbo_host, h->hist, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
    LCHK(hipStreamSynchronize(h->stream));
    if (s.numeric) return lfail(CAVI_E_NUMERIC, "sweep %d produced a non-finite value", s.call_sweeps + 1);
    return CAVI_OK;
}

cavi_status lmvb_run(lmvb_ctx *h, int32_t max_sweeps, double rel_tol, int32_t *sweeps, double *elbo)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    if (!h->ready) return lfail(CAVI_E_STATE, "lmvb_init has not run");
    if (max_sweeps < 1) return lfail(CAVI_E_INVAL, "max_sweeps=%d < 1", max_sweeps);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol)) return lfail(CAVI_E_INVAL, "rel_tol must be finite and >= 0");
    State s{};
    int done = 0, batch = 16;
    bool first = true;
    while (true) {
        const int n = std::min(batch, max_sweeps - done);
        cavi_status st = enqueue(h, n, max_sweeps, 1, rel_tol, first);
        if (st != CAVI_OK) return st;
        first = false;
        done += n;
        LCHK(hipMemcpyAsync(&s, h->st, sizeof(State), hipMemcpyDeviceToHost, h->stream));
        LCHK(hipStreamSynchronize(h->stream));
        if (s.numeric || s.converged || done >= max_sweeps) break;
        batch = std::min(batch * 2, 256);
    }
    if (sweeps) *sweeps = s.call_sweeps;
    if (elbo) *elbo = s.elbo;
    if (s.numeric) return lfail(CAVI_E_NUMERIC, "sweep %d produced a non-finite value", s.call_sweeps + 1);
    if (!s.converged) return lfail(CAVI_E_NOTCONV, "not converged after %d sweeps", s.call_sweeps);
    return CAVI_OK;
}

cavi_status lmvb_get_globals(lmvb_ctx *h, double *a_rho, double *b_rho, double *K0K, double *W, double *nu,
                             double *kappa)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    if (!h->ready) return lfail(CAVI_E_STATE, "lmvb_init has not run");
    State s;
    LCHK(hipMemcpyAsync(&s, h->st, sizeof(State), hipMemcpyDeviceToHost, h->stream));
    LCHK(hipStreamSynchronize(h->stream));
    const int M = h->sh.M;
    if (a_rho) *a_rho = s.a_rho;
    if (b_rho) *b_rho = s.b_rho;
    if (K0K)
        for (int i = 0; i < M; ++i) K0K[i] = s.K0K[i];
    if (W)
        for (int i = 0; i < M * M; ++i) W[i] = s.W[i];
    if (nu) *nu = s.nu;
    if (kappa) *kappa = s.kappa;
    return CAVI_OK;
}

cavi_status lmvb_get_genes(lmvb_ctx *h, double *m_dev, double *P_dev)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    if (!h->ready) return lfail(CAVI_E_STATE, "lmvb_init has not run");
    if ((((uintptr_t)m_dev) & 7) || (((uintptr_t)P_dev) & 7)) return lfail(CAVI_E_INVAL, "outputs must be 8-byte aligned");
    LCHK(genes_M(h->sh.M, h->sh, h->r, h->d, h->st, h->pr, m_dev, P_dev, h->stream));
    LCHK(hipStreamSynchronize(h->stream));
    return CAVI_OK;
}

cavi_status lmvb_profile_pass(lmvb_ctx *h, int32_t reps, float *ms)
{
    if (!h || !ms) return lfail(CAVI_E_INVAL, "handle or ms is NULL");
    if (!h->ready) return lfail(CAVI_E_STATE, "lmvb_init has not run");
    if (reps < 1) return lfail(CAVI_E_INVAL, "reps=%d < 1", reps);
    hipEvent_t e0, e1;
    LCHK(hipEventCreate(&e0));
    LCHK(hipEventCreate(&e1));
    // one sweep allowed, so that the pass is not skipped; the pass only writes the chunk sums,
    // which the next sweep overwrites
    hipLaunchKernelGGL(k_lm_ctl, dim3(1), dim3(1), 0, h->stream, h->st, 1, 0, 0.0);
    LCHK(hipEventRecord(e0, h->stream));
    for (int i = 0; i < reps; ++i) LCHK(pass_M(h->sh.M, h->sh, h->r, h->d, h->st, h->pr, h->partials, h->stream));
    LCHK(hipEventRecord(e1, h->stream));
    LCHK(hipEventSynchronize(e1));
    float t = 0.f;
    LCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / (float)reps;
    return CAVI_OK;
}

cavi_status lmvb_destroy(lmvb_ctx *h)
{
    if (!h) return CAVI_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->st) (void)hipFree(h->st);
    if (h->pr) (void)hipFree(h->pr);
    if (h->partials) (void)hipFree(h->partials);
    if (h->level1) (void)hipFree(h->level1);
    if (h->hist) (void)hipFree(h->hist);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return CAVI_OK;
}

}  // extern "C"
