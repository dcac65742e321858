// gfx950 kernels and C ABI (include/lmem.h) of the paper's expectation maximisation for its
// linear-mixing model (Section 4.2, eqs 42-47).
//
// One iteration is three launches:
//   k_lm_pass<M>    (linmix.h) the E-step of every gene from the current estimates: Sigma_i
//                   (eq 42), M_i (eq 43) and the gene's terms of sum M_i, sum (M_i M_i^T + Sigma_i),
//                   sum S_i (eq 44) and sum ln det Sigma_i^-1, in FP64 chunk sums of a fixed order;
//   k_lm_reduce     (linmix.h) the chunk sums in 16 contiguous groups, each in chunk order;
//   k_em_global<M>  the groups in order, the log-likelihood of the estimates the iteration started
//                   from, the M-step (eqs 45-47) and the stopping test.
// The E-step is the variational Bayes's update of q(beta_i) (eqs 20, 21) with the estimates rho,
// Lambda, Lambda K in place of E[rho], E[Lambda], E[Lambda K]: one kernel with other coefficients.
//
// Log-likelihood.  With the exact posterior of the E-step, ln p(r | theta) equals the expected
// complete-data log-likelihood plus the entropy of that posterior, both at the same theta:
//   l = -V/2 ln 2 pi + V/2 ln rho - rho/2 sum S_i + V/2 ln det Lambda
//       - 1/2 tr(Lambda sum E[(beta_i - K)(beta_i - K)^T]) + V M / 2 - 1/2 sum ln det Sigma_i^-1,
// so it comes from the sums the M-step already needs, with no per-gene logarithm.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "../../include/lmem.h"
#include "cavi_impl.h"
#include "linmix.h"

namespace {

// Estimates, their derived coefficients and the control fields of the per-call loop.
struct EmState {
    double rho;
    double K[kMaxM];
    double Lam[kMaxM * kMaxM];
    double Laminv[kMaxM * kMaxM];
    double lndetLam;
    double ll;   // log-likelihood of the estimates the last iteration started from
    double tol;
    int32_t iters, call_sweeps, max_call, stop_on_conv, converged, numeric;
    Coef coef;   // Lambda, Lambda K, rho of the next E-step
};

template <int M>
__device__ void em_coef(Coef &c, double rho, const double *Lam, const double *K)
{
    c.a_rho = 0.0;
    c.b_rho = 0.0;
    c.Erho = rho;
    for (int i = 0; i < M; ++i) {
        double t = 0.0;
        for (int j = 0; j < M; ++j) {
            c.ELam[i * M + j] = Lam[i * M + j];
            t += Lam[i * M + j] * K[j];
        }
        c.ELamK[i] = t;
    }
}

// One workgroup of 64 threads: lanes s < S add up sum s over the 16 groups in order; lane 0 does
// the rest.
template <int M>
__global__ __launch_bounds__(64) void k_em_global(Shape sh, EmState *st, const double *__restrict__ level1,
                                                  double *__restrict__ hist)
{
    if (skipped(st)) return;
    constexpr int S = M + M * (M + 1) / 2 + 2;
    __shared__ double tot[kMaxS];
    const int lane = threadIdx.x;
    if (lane < S) {
        double t = level1[lane];
        for (int b = 1; b < kGroups; ++b) t += level1[(size_t)b * kMaxS + lane];
        tot[lane] = t;
    }
    __syncthreads();
    if (lane != 0) return;
    const double V = (double)sh.V;
    const double sumS = tot[S - 2], sumlndetP = tot[S - 1];
    double K[M], Lam[M * M], Ebb[M * M];
    for (int i = 0; i < M; ++i) K[i] = st->K[i];
    for (int i = 0; i < M * M; ++i) Lam[i] = st->Lam[i];
    for (int i = 0; i < M; ++i)
        for (int k = i; k < M; ++k) {
            Ebb[i * M + k] = tot[tri(M, i, k)];
            Ebb[k * M + i] = tot[tri(M, i, k)];
        }
    // log-likelihood of the estimates this iteration started from
    const double rho = st->rho;
    double trLA = 0.0;
    for (int i = 0; i < M; ++i)
        for (int k = 0; k < M; ++k)
            trLA += Lam[i * M + k] * (Ebb[k * M + i] - tot[k] * K[i] - K[k] * tot[i] + V * K[k] * K[i]);
    const double ll = -0.5 * V * kLn2Pi + 0.5 * V * log(rho) - 0.5 * rho * sumS + 0.5 * V * st->lndetLam - 0.5 * trLA
                      + 0.5 * V * M - 0.5 * sumlndetP;
    // M-step (eqs 45-47)
    const double rho1 = V / sumS;
    double K1[M], Li1[M * M], Lam1[M * M];
    for (int i = 0; i < M; ++i) K1[i] = tot[i] / V;
    for (int i = 0; i < M; ++i)
        for (int k = 0; k < M; ++k) Li1[i * M + k] = Ebb[i * M + k] / V - K1[i] * K1[k];
    double lndetLi1 = 0.0;
    bool bad = !spd_inverse<M>(Li1, Lam1, lndetLi1);
    bad = bad || !isfinite(ll) || !isfinite(rho1) || !(rho1 > 0.0) || !isfinite(lndetLi1);
    for (int i = 0; i < M; ++i) bad = bad || !isfinite(K1[i]);
    if (bad) {
        st->numeric = 1;
        return;
    }
    const int t = st->call_sweeps + 1;
    if (t >= 2 && fabs(ll - st->ll) <= st->tol * fabs(ll)) st->converged = 1;
    hist[(t - 1) % kHistCap] = ll;
    st->ll = ll;
    st->call_sweeps = t;
    st->iters += 1;
    st->rho = rho1;
    for (int i = 0; i < M; ++i) st->K[i] = K1[i];
    for (int i = 0; i < M * M; ++i) {
        st->Lam[i] = Lam1[i];
        st->Laminv[i] = Li1[i];
    }
    st->lndetLam = -lndetLi1;
    em_coef<M>(st->coef, rho1, Lam1, K1);
}

// The E-step of the current estimates: M_i (eq 43) and Sigma_i (eq 42), one thread per gene.
template <int M>
__global__ __launch_bounds__(kThreads) void k_em_genes(Shape sh, const double *__restrict__ r,
                                                        const double *__restrict__ d, const EmState *st,
                                                        double *M_out, double *Sig_out)
{
    constexpr int N = M + 1;
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g >= sh.V) return;
    const Coef &c = st->coef;
    double dv[N], D[M], m[M], Sg[M][M], detP;
#pragma unroll
    for (int q = 0; q < N; ++q) dv[q] = d[g * N + q];
#pragma unroll
    for (int q = 0; q < M; ++q) D[q] = dv[q] - dv[N - 1];
    gene_factor<M>(D, r[g] - dv[N - 1], c, m, Sg, detP);
    if (M_out)
        for (int i = 0; i < M; ++i) M_out[g * M + i] = m[i];
    if (Sig_out)
        for (int i = 0; i < M; ++i)
            for (int k = 0; k < M; ++k) Sig_out[(g * M + i) * M + k] = Sg[i][k];
}

__global__ void k_em_ctl(EmState *st, int max_call, int stop_on_conv, double tol)
{
    st->max_call = max_call;
    st->stop_on_conv = stop_on_conv;
    st->tol = tol;
    st->call_sweeps = 0;
    st->converged = 0;
    st->numeric = 0;
}

template <int M>
hipError_t launch_iter(const Shape &sh, const double *r, const double *d, EmState *st, double *partials,
                       double *level1, double *hist, hipStream_t s)
{
    hipLaunchKernelGGL((k_lm_pass<M, false, EmState>), dim3(sh.nchunk), dim3(kThreads), 0, s, sh, r, d, st,
                       (const Prior *)nullptr, partials);
    launch_lm_reduce(sh, st, 0, partials, level1, s);
    hipLaunchKernelGGL((k_em_global<M>), dim3(1), dim3(64), 0, s, sh, st, level1, hist);
    return hipGetLastError();
}

template <int M>
hipError_t launch_epass(const Shape &sh, const double *r, const double *d, EmState *st, double *partials,
                        hipStream_t s)
{
    hipLaunchKernelGGL((k_lm_pass<M, false, EmState>), dim3(sh.nchunk), dim3(kThreads), 0, s, sh, r, d, st,
                       (const Prior *)nullptr, partials);
    return hipGetLastError();
}

template <int M>
hipError_t launch_egenes(const Shape &sh, const double *r, const double *d, const EmState *st, double *Mo,
                         double *So, hipStream_t s)
{
    const int64_t nb = (sh.V + kThreads - 1) / kThreads;
    hipLaunchKernelGGL((k_em_genes<M>), dim3((unsigned)nb), dim3(kThreads), 0, s, sh, r, d, st, Mo, So);
    return hipGetLastError();
}

// dispatch on the runtime M in [1, kMaxM]
#define EM_DISPATCH(Mrt, CALL)          \
    switch (Mrt) {                      \
    case 1: return CALL(1);             \
    case 2: return CALL(2);             \
    case 3: return CALL(3);             \
    case 4: return CALL(4);             \
    case 5: return CALL(5);             \
    case 6: return CALL(6);             \
    default: return CALL(7);            \
    }

hipError_t iter_M(const Shape &sh, const double *r, const double *d, EmState *st, double *partials, double *level1,
                  double *hist, hipStream_t s)
{
#define CALL(K) launch_iter<K>(sh, r, d, st, partials, level1, hist, s)
    EM_DISPATCH(sh.M, CALL)
#undef CALL
}

hipError_t epass_M(const Shape &sh, const double *r, const double *d, EmState *st, double *partials, hipStream_t s)
{
#define CALL(K) launch_epass<K>(sh, r, d, st, partials, s)
    EM_DISPATCH(sh.M, CALL)
#undef CALL
}

hipError_t egenes_M(const Shape &sh, const double *r, const double *d, const EmState *st, double *Mo, double *So,
                    hipStream_t s)
{
#define CALL(K) launch_egenes<K>(sh, r, d, st, Mo, So, s)
    EM_DISPATCH(sh.M, CALL)
#undef CALL
}

}  // namespace

struct lmem_ctx {
    Shape sh{};
    const double *r = nullptr, *d = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    EmState *st = nullptr;  // device
    double *partials = nullptr, *level1 = nullptr, *hist = nullptr;
};

extern "C" {

cavi_status lmem_create(lmem_ctx **out, const double *r_dev, const double *d_dev, int64_t V, int32_t N,
                        const lmem_start *start, void *hip_stream)
{
    if (!out) return lfail(CAVI_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!r_dev || !d_dev) return lfail(CAVI_E_INVAL, "r_dev or d_dev is NULL");
    if ((((uintptr_t)r_dev) & 7) || (((uintptr_t)d_dev) & 7)) return lfail(CAVI_E_INVAL, "r_dev or d_dev is not 8-byte aligned");
    if (V < 1 || V >= ((int64_t)1 << 40)) return lfail(CAVI_E_INVAL, "V=%lld outside [1, 2^40)", (long long)V);
    if (N < 2 || N > kMaxM + 1) return lfail(CAVI_E_INVAL, "N=%d outside [2, %d]", N, kMaxM + 1);
    const int M = N - 1;
    EmState s0{};
    if (start) {
        if (!start->K || !start->Lam) return lfail(CAVI_E_INVAL, "start K or Lam is NULL");
        s0.rho = start->rho;
        for (int i = 0; i < M; ++i) s0.K[i] = start->K[i];
        for (int i = 0; i < M * M; ++i) s0.Lam[i] = start->Lam[i];
    } else {
        s0.rho = 1.0;  // a0 / b0 with a0 = b0 = 0.5
        for (int i = 0; i < M; ++i) s0.K[i] = 1.0 / N;
        paper_L0(M, s0.Lam);  // n0 = 1
    }
    if (!(s0.rho > 0.0) || !isfinite(s0.rho)) return lfail(CAVI_E_INVAL, "start rho must be finite and > 0");
    for (int i = 0; i < M; ++i)
        if (!isfinite(s0.K[i])) return lfail(CAVI_E_INVAL, "start K[%d] is not finite", i);
    if (!host_spd_inverse(M, s0.Lam, s0.Laminv, &s0.lndetLam))  // ln det of its input, Lambda
        return lfail(CAVI_E_INVAL, "start Lambda is not symmetric positive definite");
    s0.coef.Erho = s0.rho;
    for (int i = 0; i < M; ++i) {
        double t = 0.0;
        for (int j = 0; j < M; ++j) {
            s0.coef.ELam[i * M + j] = s0.Lam[i * M + j];
            t += s0.Lam[i * M + j] * s0.K[j];
        }
        s0.coef.ELamK[i] = t;
    }
    lmem_ctx *h = new lmem_ctx;
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
    if ((e = hipMalloc(&h->st, sizeof(EmState))) != hipSuccess ||
        (e = hipMalloc(&h->partials, sizeof(double) * (size_t)h->sh.nchunk * h->sh.S)) != hipSuccess ||
        (e = hipMalloc(&h->level1, sizeof(double) * kGroups * kMaxS)) != hipSuccess ||
        (e = hipMalloc(&h->hist, sizeof(double) * kHistCap)) != hipSuccess) {
        (void)hipGetLastError();
        lmem_destroy(h);
        return lfail(CAVI_E_NOMEM, "device allocation: %s", hipGetErrorString(e));
    }
    e = hipMemcpyAsync(h->st, &s0, sizeof(EmState), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        lmem_destroy(h);
        return lfail(CAVI_E_HIP, "upload: %s", hipGetErrorString(e));
    }
    *out = h;
    return CAVI_OK;
}

static cavi_status em_enqueue(lmem_ctx *h, int n, int max_call, int stop_on_conv, double tol, bool begin)
{
    if (begin) hipLaunchKernelGGL(k_em_ctl, dim3(1), dim3(1), 0, h->stream, h->st, max_call, stop_on_conv, tol);
    for (int i = 0; i < n; ++i) LCHK(iter_M(h->sh, h->r, h->d, h->st, h->partials, h->level1, h->hist, h->stream));
    return CAVI_OK;
}

cavi_status lmem_iterate(lmem_ctx *h, int32_t n, double *loglik_host)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    if (n < 1 || n > kHistCap) return lfail(CAVI_E_INVAL, "n=%d outside [1, %d]", n, kHistCap);
    cavi_status st = em_enqueue(h, n, n, 0, 0.0, true);
    if (st != CAVI_OK) return st;
    EmState s;
    LCHK(hipMemcpyAsync(&s, h->st, sizeof(EmState), hipMemcpyDeviceToHost, h->stream));
    if (loglik_host) LCHK(hipMemcpyAsync(loglik_host, h->hist, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
    LCHK(hipStreamSynchronize(h->stream));
    if (s.numeric) return lfail(CAVI_E_NUMERIC, "iteration %d produced a non-finite value", s.call_sweeps + 1);
    return CAVI_OK;
}

cavi_status lmem_run(lmem_ctx *h, int32_t max_iter, double rel_tol, int32_t *iters, double *loglik)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    if (max_iter < 1) return lfail(CAVI_E_INVAL, "max_iter=%d < 1", max_iter);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol)) return lfail(CAVI_E_INVAL, "rel_tol must be finite and >= 0");
    EmState s{};
    int done = 0, batch = 16;
    bool first = true;
    while (true) {
        const int n = std::min(batch, max_iter - done);
        cavi_status st = em_enqueue(h, n, max_iter, 1, rel_tol, first);
        if (st != CAVI_OK) return st;
        first = false;
        done += n;
        LCHK(hipMemcpyAsync(&s, h->st, sizeof(EmState), hipMemcpyDeviceToHost, h->stream));
        LCHK(hipStreamSynchronize(h->stream));
        if (s.numeric || s.converged || done >= max_iter) break;
        batch = std::min(batch * 2, 256);
    }
    if (iters) *iters = s.call_sweeps;
    if (loglik) *loglik = s.ll;
    if (s.numeric) return lfail(CAVI_E_NUMERIC, "iteration %d produced a non-finite value", s.call_sweeps + 1);
    if (!s.converged) return lfail(CAVI_E_NOTCONV, "not converged after %d iterations", s.call_sweeps);
    return CAVI_OK;
}

cavi_status lmem_get_params(lmem_ctx *h, double *rho, double *K, double *Lam, double *Laminv)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    EmState s;
    LCHK(hipMemcpyAsync(&s, h->st, sizeof(EmState), hipMemcpyDeviceToHost, h->stream));
    LCHK(hipStreamSynchronize(h->stream));
    const int M = h->sh.M;
    if (rho) *rho = s.rho;
    if (K)
        for (int i = 0; i < M; ++i) K[i] = s.K[i];
    if (Lam)
        for (int i = 0; i < M * M; ++i) Lam[i] = s.Lam[i];
    if (Laminv)
        for (int i = 0; i < M * M; ++i) Laminv[i] = s.Laminv[i];
    return CAVI_OK;
}

cavi_status lmem_get_genes(lmem_ctx *h, double *M_dev, double *Sigma_dev)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    if ((((uintptr_t)M_dev) & 7) || (((uintptr_t)Sigma_dev) & 7)) return lfail(CAVI_E_INVAL, "outputs must be 8-byte aligned");
    LCHK(egenes_M(h->sh, h->r, h->d, h->st, M_dev, Sigma_dev, h->stream));
    LCHK(hipStreamSynchronize(h->stream));
    return CAVI_OK;
}

cavi_status lmem_profile_pass(lmem_ctx *h, int32_t reps, float *ms)
{
    if (!h || !ms) return lfail(CAVI_E_INVAL, "handle or ms is NULL");
    if (reps < 1) return lfail(CAVI_E_INVAL, "reps=%d < 1", reps);
    hipEvent_t e0, e1;
    LCHK(hipEventCreate(&e0));
    LCHK(hipEventCreate(&e1));
    // one iteration allowed, so that the pass is not skipped; the pass only writes the chunk sums,
    // which the next iteration overwrites
    hipLaunchKernelGGL(k_em_ctl, dim3(1), dim3(1), 0, h->stream, h->st, 1, 0, 0.0);
    LCHK(hipEventRecord(e0, h->stream));
    for (int i = 0; i < reps; ++i) LCHK(epass_M(h->sh, h->r, h->d, h->st, h->partials, h->stream));
    LCHK(hipEventRecord(e1, h->stream));
    LCHK(hipEventSynchronize(e1));
    float t = 0.f;
    LCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / (float)reps;
    return CAVI_OK;
}

cavi_status lmem_destroy(lmem_ctx *h)
{
    if (!h) return CAVI_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->st) (void)hipFree(h->st);
    if (h->partials) (void)hipFree(h->partials);
    if (h->level1) (void)hipFree(h->level1);
    if (h->hist) (void)hipFree(h->hist);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return CAVI_OK;
}

}  // extern "C"
