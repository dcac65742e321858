// Device code shared by the two inference procedures of the paper's linear-mixing model
// (Section 3.3): the variational Bayes (lmvb.hip; eqs 16-31) and the expectation maximisation
// (lmem.hip; eqs 42-47).  Both rest on the same per-gene computation: the Gaussian of beta_i given
// r_i under a precision A and a scalar c (A + c D_i D_i^T, eqs 20 and 42) and the gene's terms of
// the sums over genes that the global updates need, in FP64 with a fixed summation order.
// Included by one translation unit each; everything here has internal linkage.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <algorithm>
#include <vector>
#include "cavi_impl.h"
#include "devmath.h"
#include "../../include/cavi.h"
#include "../../include/lmvb.h"

namespace {

constexpr int kMaxM = 7;
constexpr int kThreads = 256;
constexpr int kPerThreadMax = 32;                           // genes per thread at most
constexpr int kMaxS = kMaxM + kMaxM * (kMaxM + 1) / 2 + 2;  // sums per chunk
constexpr int kGroups = 16;                                 // first-level reduction groups
constexpr int kRedThreads = 1024;
constexpr int kHistCap = 1 << 16;
constexpr double kLn2Pi = 1.8378770664093454835606594728112;
constexpr double kLnPi = 1.1447298858494001741434273513531;
constexpr double kLn2 = 0.69314718055994530941723212145818;

// Coefficients of one pass over the genes: the precision ELam and the vector ELamK of the gene
// factors, and the noise precision Erho.  The variational Bayes fills them with E[Lambda],
// E[Lambda K] and E[rho] (eqs 28, 29, 31) and keeps the q(rho) = Gamma(a_rho, b_rho) they came
// from; EM with its current Lambda, Lambda K and rho (eqs 42, 43).
struct Coef {
    double a_rho, b_rho, Erho;
    double ELam[kMaxM * kMaxM];
    double ELamK[kMaxM];
};

struct Prior {
    double a0, b0, q0, n0;
    double K0[kMaxM];
    double L0[kMaxM * kMaxM];
    double L0inv[kMaxM * kMaxM];
    double lnB0;       // ln of the Wishart prior's normaliser (0 when the prior is improper)
    double lg_a0;      // lgamma(a0)
};

struct Shape {
    int64_t V;
    int32_t N, M, nchunk, S;
    int32_t ppt;  // genes per thread: a chunk is kThreads * ppt consecutive genes
};

// position of E[beta beta^T]_{ik} (i <= k) in a chunk's sums: after the M means, row-major upper triangle
__host__ __device__ constexpr int tri(int M, int i, int k) { return M + i * M - i * (i - 1) / 2 + (k - i); }

// A state type St has the control fields below; a pass, reduction or update is skipped once the
// state has failed, used its sweeps for this call, or converged with stop-on-convergence set.
template <class St>
__device__ __forceinline__ bool skipped(const St *s)
{
    return s->numeric || s->call_sweeps >= s->max_call || (s->stop_on_conv && s->converged);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// The Gaussian of beta_i of one gene: precision P = ELam + Erho D D^T (eqs 20, 42), mean
// m = P^-1 (ELamK + Erho D e) (eqs 21, 43; e = r - mu), covariance S = P^-1, and det P.  M = 1
// and 2 use the closed-form inverse (one division); larger M factor P = L L^T, S = L^-T L^-1.
template <int M>
__device__ __forceinline__ void gene_factor(const double (&D)[M], double e, const Coef &c, double (&m)[M],
                                            double (&S)[M][M], double &detP)
{
    if constexpr (M == 1) {
        const double p = c.ELam[0] + c.Erho * D[0] * D[0];
        const double ip = 1.0 / p;
        S[0][0] = ip;
        m[0] = (c.ELamK[0] + c.Erho * D[0] * e) * ip;
        detP = p;
        return;
    }
    if constexpr (M == 2) {
        const double p00 = c.ELam[0] + c.Erho * D[0] * D[0];
        const double p01 = c.ELam[1] + c.Erho * D[0] * D[1];
        const double p11 = c.ELam[3] + c.Erho * D[1] * D[1];
        const double det = fma(p00, p11, -p01 * p01);
        const double id = 1.0 / det;
        S[0][0] = p11 * id;
        S[1][1] = p00 * id;
        S[0][1] = S[1][0] = -p01 * id;
        const double b0 = c.ELamK[0] + c.Erho * D[0] * e, b1 = c.ELamK[1] + c.Erho * D[1] * e;
        m[0] = (p11 * b0 - p01 * b1) * id;
        m[1] = (p00 * b1 - p01 * b0) * id;
        detP = det;
        return;
    }
    double L[M][M], Li[M][M], y[M];
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) L[i][j] = c.ELam[i * M + j] + c.Erho * D[i] * D[j];
    detP = 1.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double s = L[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        detP *= s;
        const double ljj = sqrt(s);
        L[j][j] = ljj;
        Li[j][j] = 1.0 / ljj;
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            double t = L[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t * Li[j][j];
        }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
        double s = c.ELamK[i] + c.Erho * D[i] * e;
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s * Li[i][i];
    }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < M; ++k) s -= L[k][i] * m[k];
        m[i] = s * Li[i][i];
    }
    // L^-1, lower triangular, by columns
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            double s = 0.0;
#pragma unroll
            for (int k = j; k < i; ++k) s -= L[i][k] * Li[k][j];
            Li[i][j] = s * Li[i][i];
        }
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = i; j < M; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = j; k < M; ++k) s += Li[k][i] * Li[k][j];
            S[i][j] = s;
            S[j][i] = s;
        }
}

// One thread per gene.  Per chunk: [sum m (M) | sum (m m^T + S) (upper triangle, row-major) |
// sum of the squared-residual bracket (eq 17 with eq 29; eq 44) | sum ln det P_i], each summed
// per thread over its genes in order (the
// log determinants as the log of their product, kept as mantissa and exponent), then over the
// wave's lanes by a fixed butterfly, then over the four waves in order.
// INIT: the gene factors of the initial state (m_i = 1/N, P_i = L0) instead of the coefficients.
template <int M, bool INIT, class St>
__global__ __launch_bounds__(kThreads) void k_lm_pass(Shape sh, const double *__restrict__ r,
                                                       const double *__restrict__ d, const St *st,
                                                       const Prior *pr, double *__restrict__ partials)
{
    constexpr int N = M + 1, S = M + M * (M + 1) / 2 + 2;
    if (!INIT && skipped(st)) return;
    __shared__ double red[kThreads / 64][S];
    const Coef c = st->coef;
    double Sinit[M][M];
    if (INIT) {
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) Sinit[i][j] = pr->L0inv[i * M + j];
    }
    double acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = 0.0;
    // product of the thread's det P_i as mantissa and binary exponent: one log per thread
    double dmant = 1.0;
    int dexp = 0;
    const int64_t g0 = (int64_t)blockIdx.x * kThreads * sh.ppt + threadIdx.x;
    for (int j = 0; j < sh.ppt; ++j) {
        const int64_t g = g0 + (int64_t)j * kThreads;
        if (g >= sh.V) break;
        double dv[N];
#pragma unroll
        for (int q = 0; q < N; ++q) dv[q] = d[g * N + q];
        const double e = r[g] - dv[N - 1];  // r_i - mu_i
        double D[M], m[M], Sg[M][M];
#pragma unroll
        for (int q = 0; q < M; ++q) D[q] = dv[q] - dv[N - 1];
        double detP = 1.0;
        if (INIT) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
                m[i] = 1.0 / N;
#pragma unroll
                for (int k = 0; k < M; ++k) Sg[i][k] = Sinit[i][k];
            }
        } else {
            gene_factor<M>(D, e, c, m, Sg, detP);
        }
        // E[beta beta^T] = m m^T + S (eq 27) and the bracket of eq 17
        double Dm = 0.0, quad = 0.0;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            acc[i] += m[i];
            Dm += D[i] * m[i];
        }
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int k = i; k < M; ++k) {
                const double ebb = m[i] * m[k] + Sg[i][k];
                acc[tri(M, i, k)] += ebb;
                quad += (i == k ? 1.0 : 2.0) * D[i] * ebb * D[k];
            }
        acc[S - 2] += e * e - 2.0 * e * Dm + quad;
        if (!INIT) {
            int e1, e2;
            const double f = frexp(detP, &e1);
            dmant = frexp(dmant * f, &e2);
            dexp += e1 + e2;
        }
    }
    acc[S - 1] = INIT ? 0.0 : log(dmant) + dexp * kLn2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const double w = wave_sum(acc[s]);
        if (lane == 0) red[wv][s] = w;
    }
    __syncthreads();
    if (threadIdx.x < S) {
        double t = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kThreads / 64; ++w) t += red[w][threadIdx.x];
        partials[(size_t)blockIdx.x * S + threadIdx.x] = t;
    }
}

// Group b sums chunks [b n / 16, (b + 1) n / 16): wave v of the NT / 64 a contiguous share of them in
// chunk order (eight loads in flight), then the waves in order.  Lane s holds sum s.
template <class St, int NT>
__global__ __launch_bounds__(NT) void k_lm_reduce(Shape sh, const St *st, int init_mode,
                                                  const double *__restrict__ partials, double *__restrict__ level1)
{
    if (!init_mode && skipped(st)) return;
    __shared__ double part[NT / 64][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = NT / 64;
    const int b = blockIdx.x;
    const int c0 = (int)(((int64_t)sh.nchunk * b) / kGroups), c1 = (int)(((int64_t)sh.nchunk * (b + 1)) / kGroups);
    const int w0 = c0 + (int)(((int64_t)(c1 - c0) * wv) / nw), w1 = c0 + (int)(((int64_t)(c1 - c0) * (wv + 1)) / nw);
    const int s = min(lane, sh.S - 1);
    double acc = 0.0;
    for (int c = w0; c < w1; c += 8) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = partials[(size_t)min(c + j, w1 - 1) * sh.S + s];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (c + j < w1) acc += v[j];
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && lane < sh.S) {
        double t = part[0][lane];
        for (int w = 1; w < nw; ++w) t += part[w][lane];
        level1[(size_t)b * kMaxS + lane] = t;
    }
}

// Up to this many chunks (V <= 65536 genes) one wave sums each group: a 1024-thread workgroup costs
// more to launch than such a group takes to add up.  The shape is a function of V only.
constexpr int kSmallReduce = 256;

template <class St>
void launch_lm_reduce(const Shape &sh, const St *st, int init_mode, const double *partials, double *level1,
                      hipStream_t s)
{
    if (sh.nchunk <= kSmallReduce)
        hipLaunchKernelGGL((k_lm_reduce<St, 64>), dim3(kGroups), dim3(64), 0, s, sh, st, init_mode, partials, level1);
    else
        hipLaunchKernelGGL((k_lm_reduce<St, kRedThreads>), dim3(kGroups), dim3(kRedThreads), 0, s, sh, st, init_mode,
                           partials, level1);
}

// Cholesky factor of an SPD M x M matrix (row-major), its inverse and ln det; false if not SPD.
template <int M>
__device__ bool spd_inverse(const double *A, double *Ainv, double &lndet)
{
    double L[M][M], Li[M][M];
    lndet = 0.0;
    for (int j = 0; j < M; ++j) {
        double s = A[j * M + j];
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        if (!(s > 0.0)) return false;
        const double ljj = sqrt(s);
        lndet += 2.0 * log(ljj);
        L[j][j] = ljj;
        Li[j][j] = 1.0 / ljj;
        for (int i = j + 1; i < M; ++i) {
            double t = A[i * M + j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t * Li[j][j];
        }
    }
    for (int j = 0; j < M; ++j)
        for (int i = j + 1; i < M; ++i) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s -= L[i][k] * Li[k][j];
            Li[i][j] = s * Li[i][i];
        }
    for (int i = 0; i < M; ++i)
        for (int j = i; j < M; ++j) {
            double s = 0.0;
            for (int k = j; k < M; ++k) s += Li[k][i] * Li[k][j];
            Ainv[i * M + j] = s;
            Ainv[j * M + i] = s;
        }
    return true;
}

cavi_status lfail(cavi_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    cavi::set_last_error(buf);
    return s;
}

#define LCHK(expr)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return lfail(CAVI_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

// Host Cholesky of an SPD matrix: inverse and ln det; false if not SPD.
bool host_spd_inverse(int M, const double *A, double *Ainv, double *lndet)
{
    std::vector<double> L(M * M, 0.0), Li(M * M, 0.0);
    double ld = 0.0;
    for (int j = 0; j < M; ++j) {
        double s = A[j * M + j];
        for (int k = 0; k < j; ++k) s -= L[j * M + k] * L[j * M + k];
        if (!(s > 0.0) || !isfinite(s)) return false;
        const double ljj = sqrt(s);
        ld += 2.0 * log(ljj);
        L[j * M + j] = ljj;
        for (int i = j + 1; i < M; ++i) {
            double t = A[i * M + j];
            if (fabs(A[i * M + j] - A[j * M + i]) > 1e-12 * (fabs(A[i * M + j]) + fabs(A[j * M + i])) + 1e-300)
                return false;  // not symmetric
            for (int k = 0; k < j; ++k) t -= L[i * M + k] * L[j * M + k];
            L[i * M + j] = t / ljj;
        }
    }
    for (int j = 0; j < M; ++j) {
        Li[j * M + j] = 1.0 / L[j * M + j];
        for (int i = j + 1; i < M; ++i) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s -= L[i * M + k] * Li[k * M + j];
            Li[i * M + j] = s / L[i * M + i];
        }
    }
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            double s = 0.0;
            for (int k = (i > j ? i : j); k < M; ++k) s += Li[k * M + i] * Li[k * M + j];
            Ainv[i * M + j] = s;
        }
    if (lndet) *lndet = ld;
    return true;
}

// Launch shape of the per-gene pass for V genes of N subpopulations: ppt genes per thread, a
// chunk of 256 ppt consecutive genes per workgroup.
Shape make_shape(int64_t V, int32_t N)
{
    Shape sh{};
    sh.V = V;
    sh.N = N;
    sh.M = N - 1;
    sh.ppt = (int32_t)std::min<int64_t>(kPerThreadMax, std::max<int64_t>(1, (V + (1 << 18) - 1) >> 18));
    const int64_t chunk = (int64_t)kThreads * sh.ppt;
    sh.nchunk = (int32_t)((V + chunk - 1) / chunk);
    sh.S = sh.M + sh.M * (sh.M + 1) / 2 + 2;
    return sh;
}

// The paper's prior scale matrix of Lambda (Section 3.5): [[0.01, 0.005], [0.005, 0.008]]^-1 for
// M = 2; the same diagonal scale, 100 I, for other M.
void paper_L0(int M, double *L0)
{
    if (M == 2) {
        const double A[4] = {0.01, 0.005, 0.005, 0.008};
        host_spd_inverse(2, A, L0, nullptr);
        return;
    }
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) L0[i * M + j] = i == j ? 100.0 : 0.0;
}

// The prior constants of eqs 5-7 from the caller's (NULL: the paper's, Section 3.5: a0 = b0 = 0.5,
// q0 = 0.001, n0 = 1, K0 = 1/N, L0 as paper_L0), with L0^-1 and ln det L0.  Returns NULL, or the
// reason the constants are invalid.
const char *fill_prior(const lmvb_prior *in, int M, Prior &p, double *lndetL0)
{
    if (in) {
        p.a0 = in->a0;
        p.b0 = in->b0;
        p.q0 = in->q0;
        p.n0 = in->n0;
        if (!in->K0 || !in->L0) return "prior K0 or L0 is NULL";
        for (int i = 0; i < M; ++i) p.K0[i] = in->K0[i];
        for (int i = 0; i < M * M; ++i) p.L0[i] = in->L0[i];
    } else {
        p.a0 = p.b0 = 0.5;
        p.q0 = 0.001;
        p.n0 = 1.0;
        for (int i = 0; i < M; ++i) p.K0[i] = 1.0 / (M + 1);
        paper_L0(M, p.L0);
    }
    for (double v : {p.a0, p.b0, p.q0, p.n0})
        if (!(v > 0.0) || !isfinite(v)) return "prior a0, b0, q0, n0 must be finite and > 0";
    for (int i = 0; i < M; ++i)
        if (!isfinite(p.K0[i])) return "prior K0 is not finite";
    if (!host_spd_inverse(M, p.L0, p.L0inv, lndetL0)) return "prior L0 is not symmetric positive definite";
    return nullptr;
}

}  // namespace
