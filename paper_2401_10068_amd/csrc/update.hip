// Global step of a sweep: fixed-order reduction of the chunk statistics, the
// conjugate updates (forms of eqs 16, 17 and 24), the lower bound (eqs
// 10-11), the convergence test, and the FP32 coefficients of the next E-step
// (expectations of eqs 26-31).
#include <math.h>

#include "cavi_impl.h"
#include "devmath.h"

namespace cavi {

namespace {

constexpr double kLn2Pi = 1.8378770664093454835606594728112;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kRedBlock = 1024;  // k_reduce: 16 waves per 64 statistics

// Sum over the 64 lanes of a wave with a fixed butterfly (same order every run).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

struct MShared {
    double red[kBlock];
    double ak[kMaxK], psi_ak[kMaxK], lg_ak[kMaxK], term_k[kMaxK];
    double tmp[kMaxKG];
    double asum, psum;
    int bad;
};

// Per-(k,g) coefficients of the E-step from one subpopulation-gene state:
//   l_nk = c_k - sum_g (h x + q)^2,  h = sqrt(E[tau]/2),  q = -m h,
//   c_k  = E ln pi_k + sum_g tmp_kg,  tmp = (E ln tau - ln 2pi - 1/beta) / 2.
__device__ __forceinline__ double coef_item(const Bufs &b, int q, double mm, double bt, double aa, double bb,
                                            double elt)
{
    const float hf = (float)sqrt(0.5 * aa / bb);
    b.hq[2 * q] = hf;
    b.hq[2 * q + 1] = (float)(-mm * (double)hf);
    b.mf[q] = (float)mm;
    return 0.5 * (elt - kLn2Pi - 1.0 / bt);
}

// c_k from the per-(k,g) parts in LDS: wave w sums subpopulations w, w+4, ...
__device__ __forceinline__ void coef_rows(const Shape &s, const Bufs &b, MShared &sh, const Prior *p,
                                          const double *T0, int with_bound)
{
    const int G = s.G, K = s.K;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = wv; k < K; k += kBlock / 64) {
        double v = 0.0;
        for (int g = lane; g < G; g += 64) v += sh.tmp[k * G + g];
        v = wave_sum(v);
        if (lane == 0) {
            const double elnpi = sh.psi_ak[k] - sh.psum;
            const double c = elnpi + v;
            b.cc[k] = (float)c;
            if (!isfinite(c)) sh.bad = 1;
            if (with_bound) {
                const double ak = sh.ak[k];
                sh.term_k[k] = T0[k] * elnpi + (p->alpha0 - 1.0) * elnpi + sh.lg_ak[k] - (ak - 1.0) * elnpi;
            }
        }
    }
}

}  // namespace

// totals[i] = sum over chunks of partials[chunk][i] in a fixed order: wave v of
// the block sums a contiguous 1/16 of the chunks (4 interleaved accumulators),
// then the 16 wave sums are added in wave order.
__global__ __launch_bounds__(kRedBlock) void k_reduce(const double *__restrict__ partials, int nchunk, int S,
                                                      double *__restrict__ totals, const Ctl *__restrict__ ctl,
                                                      int init_mode)
{
    if (!init_mode && sweep_skipped(ctl)) return;
    __shared__ double part[kRedBlock / 64][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = kRedBlock / 64;
    const int i = blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (i < S) {
        const int c0 = (int)(((int64_t)nchunk * wv) / nw), c1 = (int)(((int64_t)nchunk * (wv + 1)) / nw);
        double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
        int c = c0;
        for (; c + 4 <= c1; c += 4) {
            q0 += partials[(size_t)c * S + i];
            q1 += partials[(size_t)(c + 1) * S + i];
            q2 += partials[(size_t)(c + 2) * S + i];
            q3 += partials[(size_t)(c + 3) * S + i];
        }
        for (; c < c1; ++c) q0 += partials[(size_t)c * S + i];
        acc = (q0 + q1) + (q2 + q3);
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && i < S) {
        double t = part[0][lane];
        for (int v = 1; v < nw; ++v) t += part[v][lane];
        totals[i] = t;
    }
}

// Coefficients of the E-step from the committed state (after set_state).
__global__ __launch_bounds__(kBlock) void k_coef(Shape s, Bufs b)
{
    __shared__ MShared sh;
    const int tid = threadIdx.x, K = s.K, KG = K * s.G;
    if (tid == 0) sh.bad = 0;
    if (tid < K) sh.psi_ak[tid] = dev_digamma(b.alpha[tid]);
    for (int q = tid; q < KG; q += kBlock) {
        const double aa = b.a[q], bb = b.b[q];
        sh.tmp[q] = coef_item(b, q, b.m[q], b.beta[q], aa, bb, dev_digamma(aa) - log(bb));
    }
    __syncthreads();
    if (tid < 64) {
        double v = 0.0;
        for (int k = tid; k < K; k += 64) v += b.alpha[k];
        v = wave_sum(v);
        if (tid == 0) sh.psum = dev_digamma(v);
    }
    __syncthreads();
    coef_rows(s, b, sh, nullptr, nullptr, 0);
}

// Conjugate updates from the totals, written with sums around the E-step's
// FP32 centre c = mf:  T1 = sum r (x - c),  T2 = sum r (x - c)^2,
//   alpha = alpha0 + N_k;  beta = beta0 + N_k;  m = c + (beta0 (m0 - c) + T1) / beta;
//   a = a0 + N_k / 2;  b = b0 + [T2 + beta0 (m0 - c)^2 - beta (m - c)^2] / 2,
// then the lower bound at the new q(pi), q(mu, tau) with the entropy H of the
// responsibilities.  A non-finite value leaves the state untouched and raises
// ctl->numeric.
__global__ __launch_bounds__(kBlock) void k_mstep(Shape s, Bufs b, Prior p, int init_mode)
{
    Ctl *ctl = b.ctl;
    if (!init_mode && sweep_skipped(ctl)) return;
    __shared__ MShared sh;
    const int G = s.G, K = s.K, KG = K * G, tid = threadIdx.x;
    const double *T0 = b.totals, *T1 = T0 + K, *T2 = T1 + KG;
    const double H = T2[KG];
    if (tid == 0) sh.bad = 0;
    if (tid < K) {
        const double a = p.alpha0 + T0[tid];
        sh.ak[tid] = a;
        sh.psi_ak[tid] = dev_digamma(a);
        sh.lg_ak[tid] = dev_lgamma(a);
        b.nalpha[tid] = a;
    }
    const double half_ln_b0 = 0.5 * log(p.beta0 / kTwoPi);
    const double prior_const = half_ln_b0 + p.a0 * log(p.b0) - dev_lgamma(p.a0);
    double acc = 0.0;
    int bad = 0;
    for (int q = tid; q < KG; q += kBlock) {
        const int k = q / G, g = q - k * G;
        const double Nk = T0[k];
        const double c = (double)b.mf[q];
        const double m0p = b.m0[g] - c;
        const double bt = p.beta0 + Nk;
        const double mp = (p.beta0 * m0p + T1[q]) / bt;
        const double mm = c + mp;
        const double aa = p.a0 + 0.5 * Nk;
        double bb = p.b0 + 0.5 * (T2[q] + p.beta0 * m0p * m0p - bt * mp * mp);
        if (bb < p.b0) bb = p.b0;
        b.nm[q] = mm;
        b.nbeta[q] = bt;
        b.na[q] = aa;
        b.nb[q] = bb;
        const double elt = dev_digamma(aa) - log(bb);
        const double tb = aa / bb;
        if (!init_mode) {
            double sq = T2[q] - 2.0 * mp * T1[q] + Nk * mp * mp;  // sum r (x - m)^2
            if (sq < 0.0) sq = 0.0;
            const double dm0 = mp - m0p;                        // m - m0
            acc += 0.5 * (Nk * (elt - kLn2Pi) - tb * sq - Nk / bt);
            acc += prior_const + 0.5 * elt - 0.5 * p.beta0 * (tb * dm0 * dm0 + 1.0 / bt) + (p.a0 - 1.0) * elt
                   - p.b0 * tb;
            acc -= 0.5 * log(bt / kTwoPi) + 0.5 * elt - 0.5 + aa * log(bb) - dev_lgamma(aa) + (aa - 1.0) * elt - aa;
        }
        sh.tmp[q] = coef_item(b, q, mm, bt, aa, bb, elt);
        if (!isfinite(mm) || !isfinite(bb) || !isfinite(elt) || !isfinite(T2[q])) bad = 1;
    }
    if (bad) atomicOr(&sh.bad, 1);
    __syncthreads();
    if (tid < 64) {
        double v = 0.0;
        for (int k = tid; k < K; k += 64) v += sh.ak[k];
        v = wave_sum(v);
        if (tid == 0) {
            sh.asum = v;
            sh.psum = dev_digamma(v);
        }
    }
    __syncthreads();
    coef_rows(s, b, sh, &p, T0, !init_mode);
    sh.red[tid] = acc;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (tid < off) sh.red[tid] += sh.red[tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        if (init_mode) {
            if (!sh.bad) {
                ctl->sweeps = 0;
                ctl->call_sweeps = 0;
                ctl->converged = 0;
                ctl->numeric = 0;
                ctl->elbo = 0.0;
            } else {
                ctl->numeric = 1;
            }
        } else {
            double L = sh.red[0] + H;
            L += dev_lgamma(K * p.alpha0) - K * dev_lgamma(p.alpha0) - dev_lgamma(sh.asum);
            for (int k = 0; k < K; ++k) L += sh.term_k[k];
            if (!isfinite(L)) sh.bad = 1;
            if (sh.bad) {
                ctl->numeric = 1;
            } else {
                const int t = ctl->call_sweeps + 1;
                if (t >= 2 && fabs(L - ctl->elbo) <= ctl->tol * fabs(L)) ctl->converged = 1;
                ctl->elbo_prev = ctl->elbo;
                ctl->elbo = L;
                b.hist[(t - 1) % kHist] = L;
                ctl->call_sweeps = t;
                ctl->sweeps += 1;
            }
        }
    }
    __syncthreads();
    if (sh.bad) return;
    if (tid < K) b.alpha[tid] = b.nalpha[tid];
    for (int q = tid; q < KG; q += kBlock) {
        b.m[q] = b.nm[q];
        b.beta[q] = b.nbeta[q];
        b.a[q] = b.na[q];
        b.b[q] = b.nb[q];
    }
}

hipError_t launch_reduce(const Shape &s, const Bufs &b, int init_mode, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce, dim3((s.S + 63) / 64), dim3(kRedBlock), 0, st, b.partials, s.nchunk, s.S, b.totals,
                       b.ctl, init_mode);
    return hipGetLastError();
}

hipError_t launch_mstep(const Shape &s, const Bufs &b, const Prior &p, int init_mode, hipStream_t st)
{
    hipLaunchKernelGGL(k_mstep, dim3(1), dim3(kBlock), 0, st, s, b, p, init_mode);
    return hipGetLastError();
}

hipError_t launch_coef(const Shape &s, const Bufs &b, hipStream_t st)
{
    hipLaunchKernelGGL(k_coef, dim3(1), dim3(kBlock), 0, st, s, b);
    return hipGetLastError();
}

}  // namespace cavi
