// gfx950 kernels and C ABI (include/gibbs.h) of the paper's Gibbs sampler for its linear-mixing
// model (Section 4.1, eqs 32-40).
//
// One iteration is three launches:
//   k_gibbs_pass<M>    one thread per gene: beta_i from its full conditional (eqs 38-40) with the
//                      gene's own counter-based normals, and the gene's terms of sum beta_i,
//                      sum (beta_i - K)(beta_i - K)^T and the squared residual of eq 37, as FP64
//                      chunk sums in a fixed order (the beta_i themselves are never stored);
//   k_lm_reduce        (linmix.h) the chunk sums in 16 contiguous groups, each in chunk order;
//   k_gibbs_global<M>  the groups in order, then rho (eqs 36, 37), Lambda (eqs 32-34) and K (eq 35),
//                      the chain's row, and the coefficients of the next pass.
// Normal vectors are drawn as mean + C u with C the Cholesky factor of the covariance (the paper's
// method); the Wishart draw uses Bartlett's decomposition (O(M^2) draws, the distribution of the
// paper's sum of n0 + V + 1 outer products); Gamma draws use the Marsaglia-Tsang sampler the paper
// spells out for rho.  Everything is FP64.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "../../include/gibbs.h"
#include "cavi_impl.h"
#include "linmix.h"

namespace {

constexpr uint32_t kKey1 = 0x47494253u;
constexpr uint32_t kGlobalTag = 0x80000000u;
constexpr uint32_t kStreamRho = 1, kStreamK = 2, kStreamAOff = 3, kStreamChi = 16;
constexpr double kTwoM53 = 1.1102230246251565404236316680908203125e-16;  // 2^-53
constexpr int kMaxAttempts = 4096;  // Marsaglia-Tsang accepts with probability > 0.95 for shape >= 1
constexpr int kChainCap = 1 << 16;

struct W4 {
    uint32_t w0, w1, w2, w3;
};

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11).
__device__ __forceinline__ W4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0;
        const uint32_t h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
        const uint32_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0;
        c1 = l1;
        c2 = n2;
        c3 = l0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return W4{c0, c1, c2, c3};
}

// uniform (m + 1/2) 2^-53 from the top 53 bits of (hi lo)
__device__ __forceinline__ double u53(uint32_t lo, uint32_t hi)
{
    const uint64_t m = ((((uint64_t)hi) << 32) | lo) >> 11;
    return ((double)m + 0.5) * kTwoM53;
}

struct Block {
    double u1, u2, zc, zs;  // two uniforms and their Box-Muller pair
};

__device__ __forceinline__ Block draws(const W4 &w)
{
    Block b;
    b.u1 = u53(w.w0, w.w1);
    b.u2 = u53(w.w2, w.w3);
    const double R = sqrt(-2.0 * log(b.u1));
    // sin and cos of 2 pi u2 as sinpi and cospi of 2 u2: the same values to within rounding, with
    // an exact argument reduction instead of the general one
    double sn, cs;
    sincospi(2.0 * b.u2, &sn, &cs);
    b.zc = R * cs;
    b.zs = R * sn;
    return b;
}

__device__ __forceinline__ Block global_block(uint32_t key0, uint32_t stream, uint32_t t, uint32_t k)
{
    return draws(philox(k, 0u, t, kGlobalTag + stream, key0, kKey1));
}

// normal q of a global stream: the cosine (q even) or sine (q odd) of block q / 2
__device__ double global_normal(uint32_t key0, uint32_t stream, uint32_t t, int q)
{
    const Block b = global_block(key0, stream, t, (uint32_t)(q >> 1));
    return (q & 1) ? b.zs : b.zc;
}

// Gamma(shape, rate), shape >= 1 (Marsaglia-Tsang): attempt k takes the cosine normal of block 2k
// and the first uniform of block 2k + 1.  ok = false if no attempt is accepted within the cap.
__device__ double gamma_draw(uint32_t key0, uint32_t stream, uint32_t t, double shape, double rate, bool &ok)
{
    const double d = shape - 1.0 / 3.0, c = 1.0 / sqrt(9.0 * d);
    for (int k = 0; k < kMaxAttempts; ++k) {
        const W4 wx = philox(2u * k, 0u, t, kGlobalTag + stream, key0, kKey1);
        const W4 wu = philox(2u * k + 1u, 0u, t, kGlobalTag + stream, key0, kKey1);
        const double x = sqrt(-2.0 * log(u53(wx.w0, wx.w1))) * cospi(2.0 * u53(wx.w2, wx.w3));
        const double u = u53(wu.w0, wu.w1);
        const double w = 1.0 + c * x;
        const double v = w * w * w;
        if (v > 0.0 && log(u) < 0.5 * x * x + d - d * v + d * log(v)) return d * v / rate;
    }
    ok = false;
    return 0.0;
}

// lower Cholesky factor of an M x M SPD matrix (row-major); false if not SPD
template <int M>
__device__ bool chol(const double *A, double *L)
{
    for (int j = 0; j < M; ++j) {
        double s = A[j * M + j];
        for (int k = 0; k < j; ++k) s -= L[j * M + k] * L[j * M + k];
        if (!(s > 0.0)) return false;
        const double ljj = sqrt(s);
        L[j * M + j] = ljj;
        for (int i = j + 1; i < M; ++i) {
            double t = A[i * M + j];
            for (int k = 0; k < j; ++k) t -= L[i * M + k] * L[j * M + k];
            L[i * M + j] = t / ljj;
        }
        for (int i = 0; i < j; ++i) L[i * M + j] = 0.0;
    }
    return true;
}

struct GibbsState {
    uint32_t t;              // iterations done
    uint32_t key0;
    double rho;              // rho_t
    double K[kMaxM];         // K_{t+1}
    double Lam[kMaxM * kMaxM];  // Lambda_{t+1}
    double tol;
    int32_t call_sweeps, max_call, stop_on_conv, converged, numeric, pad;
    Coef coef;               // Lambda_{t+1}, Lambda_{t+1} K_{t+1}, rho_t: the next pass
    Coef used;               // the coefficients of iteration t's pass
};

// beta_i of gene g in iteration t: m + C z with (m, C C^T) the full conditional (eqs 38-40).
template <int M>
__device__ __forceinline__ void draw_beta(const double (&D)[M], double e, const Coef &c, uint32_t key0, uint32_t t,
                                          int64_t g, double (&beta)[M])
{
    double z[M];
#pragma unroll
    for (int j = 0; j < (M + 1) / 2; ++j) {
        const Block b = draws(philox((uint32_t)g, (uint32_t)(g >> 32), t, (uint32_t)j, key0, kKey1));
        z[2 * j] = b.zc;
        if (2 * j + 1 < M) z[2 * j + 1] = b.zs;
    }
    if constexpr (M == 1) {
        // S = 1/p, C = 1/sqrt(p)
        const double p = c.ELam[0] + c.Erho * D[0] * D[0];
        const double q = rsqrt(p);
        beta[0] = (c.ELamK[0] + c.Erho * D[0] * e) * (q * q) + q * z[0];
        return;
    }
    if constexpr (M == 2) {
        // P = [[p00, p01], [p01, p11]], S = P^-1 = [[p11, -p01], [-p01, p00]] / det; the Cholesky
        // factor of S is C11 = 1/sqrt(p11), C00 = p11 C11 / sqrt(det), C10 = -p01 C11 / sqrt(det)
        const double p00 = c.ELam[0] + c.Erho * D[0] * D[0];
        const double p01 = c.ELam[1] + c.Erho * D[0] * D[1];
        const double p11 = c.ELam[3] + c.Erho * D[1] * D[1];
        const double sd = rsqrt(fma(p00, p11, -p01 * p01));
        const double q = rsqrt(p11);
        const double id = sd * sd;
        const double b0 = c.ELamK[0] + c.Erho * D[0] * e, b1 = c.ELamK[1] + c.Erho * D[1] * e;
        const double qs = q * sd;
        beta[0] = (p11 * b0 - p01 * b1) * id + (p11 * qs) * z[0];
        beta[1] = (p00 * b1 - p01 * b0) * id - (p01 * qs) * z[0] + q * z[1];
        return;
    }
    double m[M], S[M][M], detP;
    gene_factor<M>(D, e, c, m, S, detP);
    // Cholesky factor of the covariance S, in registers
    double L[M][M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double s = S[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        const double ljj = sqrt(s);
        L[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            double t2 = S[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) t2 -= L[i][k] * L[j][k];
            L[i][j] = t2 / ljj;
        }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
        double s = m[i];
#pragma unroll
        for (int k = 0; k <= i; ++k) s += L[i][k] * z[k];
        beta[i] = s;
    }
}

// One thread per gene.  Per chunk: [sum beta (M) | sum (beta - K)(beta - K)^T (upper triangle,
// row-major) | sum of squared residuals], each summed per thread over its genes in order, then over
// the wave by a fixed butterfly, then over the four waves in order.
template <int M>
__global__ __launch_bounds__(kThreads) void k_gibbs_pass(Shape sh, const double *__restrict__ r,
                                                          const double *__restrict__ d, const GibbsState *st,
                                                          double *__restrict__ partials)
{
    constexpr int N = M + 1, S = M + M * (M + 1) / 2 + 1;
    if (skipped(st)) return;
    __shared__ double red[kThreads / 64][S];
    const Coef c = st->coef;
    const uint32_t key0 = st->key0, t = st->t + 1;
    double K[M];
#pragma unroll
    for (int i = 0; i < M; ++i) K[i] = st->K[i];
    double acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = 0.0;
    const int64_t g0 = (int64_t)blockIdx.x * kThreads * sh.ppt + threadIdx.x;
    for (int j = 0; j < sh.ppt; ++j) {
        const int64_t g = g0 + (int64_t)j * kThreads;
        if (g >= sh.V) break;
        double dv[N];
#pragma unroll
        for (int q = 0; q < N; ++q) dv[q] = d[g * N + q];
        const double e = r[g] - dv[N - 1];
        double D[M], beta[M];
#pragma unroll
        for (int q = 0; q < M; ++q) D[q] = dv[q] - dv[N - 1];
        draw_beta<M>(D, e, c, key0, t, g, beta);
        double res = e, db[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
            acc[i] += beta[i];
            res -= D[i] * beta[i];
            db[i] = beta[i] - K[i];
        }
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int k = i; k < M; ++k) acc[tri(M, i, k)] += db[i] * db[k];
        acc[S - 1] += res * res;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const double w = wave_sum(acc[s]);
        if (lane == 0) red[wv][s] = w;
    }
    __syncthreads();
    if (threadIdx.x < S) {
        double tot = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kThreads / 64; ++w) tot += red[w][threadIdx.x];
        partials[(size_t)blockIdx.x * S + threadIdx.x] = tot;
    }
}

// One workgroup of four waves, each on its own SIMD, so that independent work overlaps:
//   wave 0: lanes s < S add up sum s over the 16 groups in order; lane 0 gathers them and forms the
//           Cholesky factor of the Wishart scale Lambda_L^-1 (eqs 32-34 with K_t; no draw needed);
//   wave 1: lanes 0..M-1 the chi-square variates of Bartlett's diagonal, lane M rho_t (its rate
//           from the same group sums in the same order);
//   wave 2: the below-diagonal normals of Bartlett's factor, then the normals of K_{t+1}.
// Then wave 0's lane 0 forms Lambda_{t+1} and K_{t+1} and writes row t of the chain
// (rho_t, K_t, Lambda_t).  A failed Gamma draw is recorded as -1.
template <int M>
__global__ __launch_bounds__(256) void k_gibbs_global(Shape sh, GibbsState *st, const Prior *pr,
                                                      const double *__restrict__ level1, double *__restrict__ chain)
{
    if (skipped(st)) return;
    constexpr int S = M + M * (M + 1) / 2 + 1, R = 1 + M + M * M, NOFF = M * (M - 1) / 2;
    static_assert(S <= 64 && M + 1 <= 64 && NOFF + M <= 64, "one wave per kind of work");
    __shared__ double gam[kMaxM + 1], zn[kMaxM * (kMaxM - 1) / 2 + kMaxM];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double V = (double)sh.V;
    const uint32_t key0 = st->key0, t = st->t + 1;
    const double n = pr->n0 + V + 1.0;
    double tot[S], K[M], Lc[M * M];
    bool ok = true;
    if (wv == 0) {
        double v = 0.0;
        if (lane < S) {
            v = level1[lane];
            for (int b = 1; b < kGroups; ++b) v += level1[(size_t)b * kMaxS + lane];
        }
#pragma unroll
        for (int q = 0; q < S; ++q) tot[q] = __shfl(v, q, 64);
        if (lane == 0) {
            // Lambda_L (eq 34) with K_t, and the Cholesky factor of its inverse
            double LamL[M * M], Sc[M * M], lnd;
            for (int i = 0; i < M; ++i) K[i] = st->K[i];
            for (int i = 0; i < M; ++i)
                for (int k = 0; k < M; ++k) {
                    const int a = i < k ? i : k, b = i < k ? k : i;
                    LamL[i * M + k] =
                        pr->L0inv[i * M + k] + pr->q0 * (K[i] - pr->K0[i]) * (K[k] - pr->K0[k]) + tot[tri(M, a, b)];
                }
            ok = spd_inverse<M>(LamL, Sc, lnd) && chol<M>(Sc, Lc);
        }
    } else if (wv == 1) {
        if (lane <= M) {
            double shape = 0.5 * (n - lane), rate = 0.5;
            uint32_t stream = kStreamChi + lane, tt = t + 1;
            if (lane == M) {  // rho_t (eqs 36, 37)
                double res = level1[S - 1];
                for (int b = 1; b < kGroups; ++b) res += level1[(size_t)b * kMaxS + S - 1];
                shape = pr->a0 + 0.5 * V;
                rate = pr->b0 + 0.5 * res;
                stream = kStreamRho;
                tt = t;
            }
            bool gok = true;
            const double g = gamma_draw(key0, stream, tt, shape, rate, gok);
            gam[lane] = gok ? g : -1.0;
        }
    } else if (wv == 2) {
        if (lane < NOFF + M) {
            const bool off = lane < NOFF;
            zn[lane] = global_normal(key0, off ? kStreamAOff : kStreamK, t + 1, off ? lane : lane - NOFF);
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double rho = gam[M];
    ok = ok && rho > 0.0;
    for (int i = 0; i < M; ++i) ok = ok && gam[i] > 0.0;
    // Lambda_{t+1} by Bartlett's decomposition of Wishart(n, LamL^-1)
    double A[M * M];
    int q = 0;
    for (int i = 0; i < M; ++i) {
        for (int j = 0; j < M; ++j) A[i * M + j] = 0.0;
        A[i * M + i] = sqrt(gam[i]);
        for (int j = 0; j < i; ++j) A[i * M + j] = zn[q++];
    }
    double LA[M * M], Lam1[M * M], lnd;
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            double s = 0.0;
            for (int k = j; k <= i; ++k) s += Lc[i * M + k] * A[k * M + j];  // both lower triangular
            LA[i * M + j] = s;
        }
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            double s = 0.0;
            for (int k = 0; k < M; ++k) s += LA[i * M + k] * LA[j * M + k];
            Lam1[i * M + j] = s;
        }
    // K_{t+1} (eq 35): mean + C u, C the Cholesky factor of ((q0 + V) Lambda_{t+1})^-1
    double P[M * M], Cv[M * M], Ck[M * M], K1[M];
    for (int i = 0; i < M * M; ++i) P[i] = (pr->q0 + V) * Lam1[i];
    ok = ok && spd_inverse<M>(P, Cv, lnd) && chol<M>(Cv, Ck);
    for (int i = 0; i < M; ++i) {
        double s = (pr->q0 * pr->K0[i] + tot[i]) / (pr->q0 + V);
        for (int k = 0; k <= i; ++k) s += Ck[i * M + k] * zn[NOFF + k];
        K1[i] = s;
    }
    ok = ok && isfinite(rho) && rho > 0.0;
    for (int i = 0; i < M; ++i) ok = ok && isfinite(K1[i]);
    for (int i = 0; i < M * M; ++i) ok = ok && isfinite(Lam1[i]);
    if (!ok) {
        st->numeric = 1;
        return;
    }
    // row t: rho_t, K_t, Lambda_t
    double *row = chain + (size_t)((t - 1) % kChainCap) * R;
    row[0] = rho;
    for (int i = 0; i < M; ++i) row[1 + i] = K[i];
    for (int i = 0; i < M * M; ++i) row[1 + M + i] = st->Lam[i];
    st->used = st->coef;
    st->t = t;
    st->call_sweeps += 1;
    st->rho = rho;
    for (int i = 0; i < M; ++i) st->K[i] = K1[i];
    for (int i = 0; i < M * M; ++i) st->Lam[i] = Lam1[i];
    Coef &c = st->coef;
    c.Erho = rho;
    for (int i = 0; i < M; ++i) {
        double s = 0.0;
        for (int j = 0; j < M; ++j) {
            c.ELam[i * M + j] = Lam1[i * M + j];
            s += Lam1[i * M + j] * K1[j];
        }
        c.ELamK[i] = s;
    }
}

template <int M>
__global__ __launch_bounds__(kThreads) void k_gibbs_genes(Shape sh, const double *__restrict__ r,
                                                           const double *__restrict__ d, const GibbsState *st,
                                                           double *beta_out)
{
    constexpr int N = M + 1;
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g >= sh.V) return;
    double dv[N], D[M], beta[M];
#pragma unroll
    for (int q = 0; q < N; ++q) dv[q] = d[g * N + q];
#pragma unroll
    for (int q = 0; q < M; ++q) D[q] = dv[q] - dv[N - 1];
    draw_beta<M>(D, r[g] - dv[N - 1], st->used, st->key0, st->t, g, beta);
    for (int i = 0; i < M; ++i) beta_out[g * M + i] = beta[i];
}

__global__ void k_gibbs_ctl(GibbsState *st, int max_call)
{
    st->max_call = max_call;
    st->stop_on_conv = 0;
    st->call_sweeps = 0;
    st->converged = 0;
    st->numeric = 0;
}

template <int M>
hipError_t launch_giter(const Shape &sh, const double *r, const double *d, GibbsState *st, const Prior *pr,
                        double *partials, double *level1, double *chain, hipStream_t s)
{
    hipLaunchKernelGGL((k_gibbs_pass<M>), dim3(sh.nchunk), dim3(kThreads), 0, s, sh, r, d, st, partials);
    launch_lm_reduce(sh, st, 0, partials, level1, s);
    hipLaunchKernelGGL((k_gibbs_global<M>), dim3(1), dim3(256), 0, s, sh, st, pr, level1, chain);
    return hipGetLastError();
}

template <int M>
hipError_t launch_gpass(const Shape &sh, const double *r, const double *d, GibbsState *st, double *partials,
                        hipStream_t s)
{
    hipLaunchKernelGGL((k_gibbs_pass<M>), dim3(sh.nchunk), dim3(kThreads), 0, s, sh, r, d, st, partials);
    return hipGetLastError();
}

template <int M>
hipError_t launch_ggenes(const Shape &sh, const double *r, const double *d, const GibbsState *st, double *beta,
                         hipStream_t s)
{
    const int64_t nb = (sh.V + kThreads - 1) / kThreads;
    hipLaunchKernelGGL((k_gibbs_genes<M>), dim3((unsigned)nb), dim3(kThreads), 0, s, sh, r, d, st, beta);
    return hipGetLastError();
}

// dispatch on the runtime M in [1, kMaxM]
#define G_DISPATCH(Mrt, CALL)  \
    switch (Mrt) {             \
    case 1: return CALL(1);    \
    case 2: return CALL(2);    \
    case 3: return CALL(3);    \
    case 4: return CALL(4);    \
    case 5: return CALL(5);    \
    case 6: return CALL(6);    \
    default: return CALL(7);   \
    }

hipError_t giter_M(const Shape &sh, const double *r, const double *d, GibbsState *st, const Prior *pr, double *partials,
                   double *level1, double *chain, hipStream_t s)
{
#define CALL(K) launch_giter<K>(sh, r, d, st, pr, partials, level1, chain, s)
    G_DISPATCH(sh.M, CALL)
#undef CALL
}

hipError_t gpass_M(const Shape &sh, const double *r, const double *d, GibbsState *st, double *partials, hipStream_t s)
{
#define CALL(K) launch_gpass<K>(sh, r, d, st, partials, s)
    G_DISPATCH(sh.M, CALL)
#undef CALL
}

hipError_t ggenes_M(const Shape &sh, const double *r, const double *d, const GibbsState *st, double *beta,
                    hipStream_t s)
{
#define CALL(K) launch_ggenes<K>(sh, r, d, st, beta, s)
    G_DISPATCH(sh.M, CALL)
#undef CALL
}

}  // namespace

struct gibbs_ctx {
    Shape sh{};
    const double *r = nullptr, *d = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    GibbsState *st = nullptr;  // device
    Prior *pr = nullptr;       // device
    double *partials = nullptr, *level1 = nullptr, *chain = nullptr;
    uint32_t t = 0;            // iterations done (host copy)
};

extern "C" {

cavi_status gibbs_create(gibbs_ctx **out, const double *r_dev, const double *d_dev, int64_t V, int32_t N,
                         const lmvb_prior *prior, uint64_t seed, void *hip_stream)
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
    if (!(p.n0 + (double)V >= M)) return lfail(CAVI_E_INVAL, "n0 + V must be at least N - 1 (Wishart draws)");
    if (!(p.a0 + 0.5 * (double)V >= 1.0)) return lfail(CAVI_E_INVAL, "a0 + V/2 must be at least 1 (Gamma draws)");
    GibbsState s0{};
    s0.t = 0;
    s0.key0 = (uint32_t)seed;
    s0.rho = p.a0 / p.b0;
    for (int i = 0; i < M; ++i) s0.K[i] = p.K0[i];
    for (int i = 0; i < M * M; ++i) s0.Lam[i] = p.n0 * p.L0[i];
    s0.coef.Erho = s0.rho;
    for (int i = 0; i < M; ++i) {
        double t = 0.0;
        for (int j = 0; j < M; ++j) {
            s0.coef.ELam[i * M + j] = s0.Lam[i * M + j];
            t += s0.Lam[i * M + j] * s0.K[j];
        }
        s0.coef.ELamK[i] = t;
    }
    gibbs_ctx *h = new gibbs_ctx;
    h->sh = make_shape(V, N);
    h->sh.S = M + M * (M + 1) / 2 + 1;
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
    const size_t R = 1 + M + (size_t)M * M;
    if ((e = hipMalloc(&h->st, sizeof(GibbsState))) != hipSuccess || (e = hipMalloc(&h->pr, sizeof(Prior))) != hipSuccess ||
        (e = hipMalloc(&h->partials, sizeof(double) * (size_t)h->sh.nchunk * h->sh.S)) != hipSuccess ||
        (e = hipMalloc(&h->level1, sizeof(double) * kGroups * kMaxS)) != hipSuccess ||
        (e = hipMalloc(&h->chain, sizeof(double) * kChainCap * R)) != hipSuccess) {
        (void)hipGetLastError();
        gibbs_destroy(h);
        return lfail(CAVI_E_NOMEM, "device allocation: %s", hipGetErrorString(e));
    }
    e = hipMemcpyAsync(h->pr, &p, sizeof(Prior), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h->st, &s0, sizeof(GibbsState), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        gibbs_destroy(h);
        return lfail(CAVI_E_HIP, "upload: %s", hipGetErrorString(e));
    }
    *out = h;
    return CAVI_OK;
}

cavi_status gibbs_iterate(gibbs_ctx *h, int32_t n)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    if (n < 1) return lfail(CAVI_E_INVAL, "n=%d < 1", n);
    if ((uint64_t)h->t + (uint64_t)n > 0xFFFFFFFEull) return lfail(CAVI_E_INVAL, "at most 2^32 - 2 iterations");
    hipLaunchKernelGGL(k_gibbs_ctl, dim3(1), dim3(1), 0, h->stream, h->st, n);
    for (int i = 0; i < n; ++i)
        LCHK(giter_M(h->sh, h->r, h->d, h->st, h->pr, h->partials, h->level1, h->chain, h->stream));
    GibbsState s;
    LCHK(hipMemcpyAsync(&s, h->st, sizeof(GibbsState), hipMemcpyDeviceToHost, h->stream));
    LCHK(hipStreamSynchronize(h->stream));
    h->t = s.t;
    if (s.numeric) return lfail(CAVI_E_NUMERIC, "iteration %u produced a non-finite value or an indefinite matrix", s.t + 1);
    return CAVI_OK;
}

cavi_status gibbs_get_chain(gibbs_ctx *h, int64_t first, int32_t count, double *rho, double *K, double *Lam)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    if (count < 1 || first < 0 || first + count > (int64_t)h->t || (int64_t)h->t - first > kChainCap)
        return lfail(CAVI_E_INVAL, "rows [%lld, %lld) not available (%u drawn, the last %d kept)", (long long)first,
                     (long long)(first + count), h->t, kChainCap);
    const int M = h->sh.M;
    const size_t R = 1 + M + (size_t)M * M;
    std::vector<double> buf((size_t)count * R);
    int64_t done = 0;
    while (done < count) {  // the ring may wrap once
        const int64_t row = first + done, slot = row % kChainCap;
        const int64_t n = std::min<int64_t>(count - done, kChainCap - slot);
        LCHK(hipMemcpyAsync(buf.data() + done * R, h->chain + slot * R, sizeof(double) * n * R, hipMemcpyDeviceToHost,
                            h->stream));
        done += n;
    }
    LCHK(hipStreamSynchronize(h->stream));
    for (int32_t i = 0; i < count; ++i) {
        const double *x = buf.data() + (size_t)i * R;
        if (rho) rho[i] = x[0];
        if (K)
            for (int k = 0; k < M; ++k) K[(size_t)i * M + k] = x[1 + k];
        if (Lam)
            for (int k = 0; k < M * M; ++k) Lam[(size_t)i * M * M + k] = x[1 + M + k];
    }
    return CAVI_OK;
}

cavi_status gibbs_get_state(gibbs_ctx *h, int64_t *t, double *rho, double *K, double *Lam)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    GibbsState s;
    LCHK(hipMemcpyAsync(&s, h->st, sizeof(GibbsState), hipMemcpyDeviceToHost, h->stream));
    LCHK(hipStreamSynchronize(h->stream));
    const int M = h->sh.M;
    if (t) *t = s.t;
    if (rho) *rho = s.rho;
    if (K)
        for (int i = 0; i < M; ++i) K[i] = s.K[i];
    if (Lam)
        for (int i = 0; i < M * M; ++i) Lam[i] = s.Lam[i];
    return CAVI_OK;
}

cavi_status gibbs_get_genes(gibbs_ctx *h, double *beta_dev)
{
    if (!h) return lfail(CAVI_E_INVAL, "handle is NULL");
    if (!beta_dev || (((uintptr_t)beta_dev) & 7)) return lfail(CAVI_E_INVAL, "beta_dev is NULL or not 8-byte aligned");
    if (h->t == 0) return lfail(CAVI_E_STATE, "no iteration yet");
    LCHK(ggenes_M(h->sh, h->r, h->d, h->st, beta_dev, h->stream));
    LCHK(hipStreamSynchronize(h->stream));
    return CAVI_OK;
}

cavi_status gibbs_profile_pass(gibbs_ctx *h, int32_t reps, float *ms)
{
    if (!h || !ms) return lfail(CAVI_E_INVAL, "handle or ms is NULL");
    if (reps < 1) return lfail(CAVI_E_INVAL, "reps=%d < 1", reps);
    hipEvent_t e0, e1;
    LCHK(hipEventCreate(&e0));
    LCHK(hipEventCreate(&e1));
    // one iteration allowed, so that the pass is not skipped; the pass only writes the chunk sums,
    // which the next iteration overwrites
    hipLaunchKernelGGL(k_gibbs_ctl, dim3(1), dim3(1), 0, h->stream, h->st, 1);
    LCHK(hipEventRecord(e0, h->stream));
    for (int i = 0; i < reps; ++i) LCHK(gpass_M(h->sh, h->r, h->d, h->st, h->partials, h->stream));
    LCHK(hipEventRecord(e1, h->stream));
    LCHK(hipEventSynchronize(e1));
    float t = 0.f;
    LCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / (float)reps;
    return CAVI_OK;
}

cavi_status gibbs_destroy(gibbs_ctx *h)
{
    if (!h) return CAVI_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->st) (void)hipFree(h->st);
    if (h->pr) (void)hipFree(h->pr);
    if (h->partials) (void)hipFree(h->partials);
    if (h->level1) (void)hipFree(h->level1);
    if (h->chain) (void)hipFree(h->chain);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return CAVI_OK;
}

}  // extern "C"
