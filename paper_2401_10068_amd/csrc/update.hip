// Global step of a sweep, per dataset: fixed-order reduction of the chunk
// statistics, the conjugate updates (forms of eqs 16, 17 and 24), the lower
// bound (eqs 10-11), the convergence test, and the FP32 coefficients of the
// next E-step (expectations of eqs 26-31).
#include <math.h>

#include "cavi_impl.h"
#include "devmath.h"

namespace cavi {

namespace {

constexpr double kLn2Pi = 1.8378770664093454835606594728112;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kRedBlock = 1024;  // k_reduce: 16 waves per 64 statistics
constexpr int kMBlock = 1024;    // k_mstep, k_coef: one (k, g) item per thread up to K G = 1024

// Sum over the 64 lanes of a wave with a fixed butterfly (same order every run).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

struct MShared {
    double red[kMBlock / 64];
    double ak[kMaxK], psi_ak[kMaxK], lg_ak[kMaxK], term_k[kMaxK], nk[kMaxK];
    double psi_a[kMaxK], lg_a[kMaxK], ln_bt[kMaxK];  // per component: digamma, lgamma of a_kg; ln(beta_kg / 2 pi)
    double tmp[kMaxKG];
    double asum, psum, lg_asum, lg_prior;
    int bad;
};

// Per-dataset views of the batch arrays.
struct View {
    int K, G;
    double *alpha, *m, *beta, *a, *b;
    double *nalpha, *nm, *nbeta, *na, *nb;
    const double *m0;
    float *cc, *hq, *mf;
    const double *totals;  // nsplit x smax: the sums of the dataset's chunk ranges
    size_t smax;
    int nsplit;
    double *hist;
    Ctl *ctl;
};

__device__ __forceinline__ View view(const Shape &s, const Bufs &bf, int bi)
{
    View v;
    const size_t kb = (size_t)bi * s.Kmax, kg = kb * s.G;
    v.K = bf.ds[bi].K;
    v.G = s.G;
    v.alpha = bf.alpha + kb;
    v.nalpha = bf.nalpha + kb;
    v.m = bf.m + kg;
    v.beta = bf.beta + kg;
    v.a = bf.a + kg;
    v.b = bf.b + kg;
    v.nm = bf.nm + kg;
    v.nbeta = bf.nbeta + kg;
    v.na = bf.na + kg;
    v.nb = bf.nb + kg;
    v.m0 = bf.m0 + (size_t)bi * s.G;
    v.cc = bf.cc + kb;
    v.hq = bf.hq + 2 * kg;
    v.mf = bf.mf + kg;
    v.totals = bf.totals + (size_t)bi * red_split_max(s.Nmax) * s.Smax;
    v.smax = (size_t)s.Smax;
    v.nsplit = red_split(bf.ds[bi].nchunk);
    v.hist = bf.hist + (size_t)bi * s.hist_cap;
    v.ctl = bf.ctl + bi;
    return v;
}

// Statistic i of the dataset: the sums of its chunk ranges, added in range order.
__device__ __forceinline__ double total(const View &v, int i)
{
    double t = v.totals[i];
    if (v.nsplit > 1) {  // kRedSplit ranges: their loads issued together
#pragma unroll
        for (int z = 1; z < kRedSplit; ++z) t += v.totals[z * v.smax + i];
    }
    return t;
}

// Per-(k,g) coefficients of the E-step from one subpopulation-gene state:
//   l_nk = c_k - sum_g (h x + q)^2,  h = sqrt(E[tau]/2),  q = -m h,
//   c_k  = E ln pi_k + sum_g tmp_kg,  tmp = (E ln tau - ln 2pi - 1/beta) / 2.
__device__ __forceinline__ double coef_item(const View &v, int q, double mm, double bt, double aa, double bb,
                                            double elt)
{
    const float hf = (float)sqrt(0.5 * aa / bb);
    v.hq[2 * q] = hf;
    v.hq[2 * q + 1] = (float)(-mm * (double)hf);
    v.mf[q] = (float)mm;
    return 0.5 * (elt - kLn2Pi - 1.0 / bt);
}

// c_k from the per-(k,g) parts in LDS: wave w sums subpopulations w, w+16, ...
__device__ __forceinline__ void coef_rows(const View &v, MShared &sh, const Prior *p, int with_bound)
{
    const int G = v.G, K = v.K;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = wv; k < K; k += kMBlock / 64) {
        double x = 0.0;
        for (int g = lane; g < G; g += 64) x += sh.tmp[k * G + g];
        x = wave_sum(x);
        if (lane == 0) {
            const double elnpi = sh.psi_ak[k] - sh.psum;
            const double c = elnpi + x;
            v.cc[k] = (float)c;
            if (!isfinite(c)) sh.bad = 1;
            if (with_bound) {
                const double ak = sh.ak[k];
                sh.term_k[k] = sh.nk[k] * elnpi + (p->alpha0 - 1.0) * elnpi + sh.lg_ak[k] - (ak - 1.0) * elnpi;
            }
        }
    }
}

}  // namespace

// totals[b][z][i] = sum over the chunks of range z of dataset b (its chunks [z n / Z, (z + 1) n / Z)
// for Z = red_split(n)) of partials[chunk][i], in a fixed order: wave v of the block sums a
// contiguous 1/16 of the range's chunks (4 interleaved accumulators), then the 16 wave sums are added
// in wave order.  The ranges spread a large dataset over Z workgroups per 64 statistics; the update
// adds them.
__global__ __launch_bounds__(kRedBlock) void k_reduce(Shape s, Bufs bf, int init_mode)
{
    __shared__ double part[kRedBlock / 64][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = kRedBlock / 64;
    const int i = blockIdx.x * 64 + lane;
    const int z = blockIdx.z;
    const int nds = n_active_datasets(s, bf);
    for (int slot = blockIdx.y; slot < nds; slot += gridDim.y) {
        const int bi = active_dataset(s, bf, slot);
        if (!init_mode && sweep_skipped(bf.ctl + bi)) continue;
        const Ds d = bf.ds[bi];
        const int S = d.K + 2 * d.K * s.G + 1;
        if (blockIdx.x * 64 >= S) continue;
        const int Z = red_split(d.nchunk);
        if (z >= Z) continue;
        const int r0 = (int)(((int64_t)d.nchunk * z) / Z), r1 = (int)(((int64_t)d.nchunk * (z + 1)) / Z);
        const double *pp = bf.partials + (size_t)(d.chunk0 + r0) * s.Smax;
        const int nr = r1 - r0;
        double acc = 0.0;
        if (i < S) {
            const int c0 = (int)(((int64_t)nr * wv) / nw), c1 = (int)(((int64_t)nr * (wv + 1)) / nw);
            double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
            int c = c0;
            for (; c + 4 <= c1; c += 4) {
                q0 += pp[(size_t)c * s.Smax + i];
                q1 += pp[(size_t)(c + 1) * s.Smax + i];
                q2 += pp[(size_t)(c + 2) * s.Smax + i];
                q3 += pp[(size_t)(c + 3) * s.Smax + i];
            }
            for (; c < c1; ++c) q0 += pp[(size_t)c * s.Smax + i];
            acc = (q0 + q1) + (q2 + q3);
        }
        part[wv][lane] = acc;
        __syncthreads();
        if (wv == 0 && i < S) {
            double t = part[0][lane];
            for (int v = 1; v < nw; ++v) t += part[v][lane];
            bf.totals[((size_t)bi * red_split_max(s.Nmax) + z) * s.Smax + i] = t;
        }
        __syncthreads();  // part is rewritten by the next dataset
    }
}

// Coefficients of the E-step from the committed state (after set_state).
__global__ __launch_bounds__(kMBlock) void k_coef(Shape s, Bufs bf)
{
    __shared__ MShared sh;
    const View v = view(s, bf, blockIdx.x);
    const int tid = threadIdx.x, K = v.K, KG = K * v.G;
    if (tid == 0) sh.bad = 0;
    if (tid < K) sh.psi_ak[tid] = dev_digamma(v.alpha[tid]);
    for (int q = tid; q < KG; q += kMBlock) {
        const double aa = v.a[q], bb = v.b[q];
        sh.tmp[q] = coef_item(v, q, v.m[q], v.beta[q], aa, bb, dev_digamma(aa) - log(bb));
    }
    __syncthreads();
    if (tid < 64) {
        double x = 0.0;
        for (int k = tid; k < K; k += 64) x += v.alpha[k];
        x = wave_sum(x);
        if (tid == 0) sh.psum = dev_digamma(x);
    }
    __syncthreads();
    coef_rows(v, sh, nullptr, 0);
}

// Conjugate updates from the totals, written with sums around the E-step's
// FP32 centre c = mf:  T1 = sum r (x - c),  T2 = sum r (x - c)^2,
//   alpha = alpha0 + N_k;  beta = beta0 + N_k;  m = c + (beta0 (m0 - c) + T1) / beta;
//   a = a0 + N_k / 2;  b = b0 + [T2 + beta0 (m0 - c)^2 - beta (m - c)^2] / 2,
// then the lower bound at the new q(pi), q(mu, tau) with the entropy H of the
// responsibilities.  A non-finite value leaves the state untouched and raises
// ctl->numeric.
__device__ __forceinline__ void mstep_one(const Shape &s, const Bufs &bf, const Prior &p, int init_mode, int bi,
                                          MShared &sh)
{
    const View v = view(s, bf, bi);
    Ctl *ctl = v.ctl;
    if (!init_mode && sweep_skipped(ctl)) return;
    const int G = v.G, K = v.K, KG = K * G, tid = threadIdx.x;
    if (tid == 0) sh.bad = 0;
    if (tid < K) {
        const double nk = total(v, tid);
        sh.nk[tid] = nk;
        const double a = p.alpha0 + nk;
        sh.ak[tid] = a;
        sh.psi_ak[tid] = dev_digamma(a);
        sh.lg_ak[tid] = dev_lgamma(a);
        v.nalpha[tid] = a;
    } else if (tid >= 64 && tid < 64 + K) {
        // a_kg = a0 + N_k / 2 and beta_kg = beta0 + N_k are the same for every gene of a
        // subpopulation: their special functions once per subpopulation, in other waves
        const int k = tid - 64;
        const double nk = total(v, k);
        sh.psi_a[k] = dev_digamma(p.a0 + 0.5 * nk);
        sh.ln_bt[k] = log((p.beta0 + nk) / kTwoPi);
    } else if (tid >= 128 && tid < 128 + K) {
        const int k = tid - 128;
        sh.lg_a[k] = dev_lgamma(p.a0 + 0.5 * total(v, k));
    } else if ((tid >= 192 && tid < 256) || (!init_mode && tid >= 256 && tid < 320)) {
        // digamma (wave 3) and lgamma (wave 4) of sum(alpha), whose terms are known already
        double x = 0.0;
        for (int k = tid & 63; k < K; k += 64) x += p.alpha0 + total(v, k);
        x = wave_sum(x);
        if (tid == 192) {
            sh.asum = x;
            sh.psum = dev_digamma(x);
        }
        if (tid == 256) sh.lg_asum = dev_lgamma(x);
    } else if (!init_mode && tid == 320) {
        sh.lg_prior = dev_lgamma(K * p.alpha0) - K * dev_lgamma(p.alpha0);
    }
    __syncthreads();
    const double half_ln_b0 = 0.5 * log(p.beta0 / kTwoPi);
    const double prior_const = half_ln_b0 + p.a0 * log(p.b0) - dev_lgamma(p.a0);
    double acc = 0.0;
    int bad = 0;
    // the new state of this thread's items stays in registers until the commit
    constexpr int kItems = kMaxKG / kMBlock;
    double nmv[kItems], nbt[kItems], nav[kItems], nbv[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int q = tid + it * kMBlock;
        if (q >= KG) break;
        const int k = q / G, g = q - k * G;
        const double Nk = sh.nk[k];
        const double T1q = total(v, K + q), T2q = total(v, K + KG + q);
        const double c = (double)v.mf[q];
        const double m0p = v.m0[g] - c;
        const double bt = p.beta0 + Nk;
        const double mp = (p.beta0 * m0p + T1q) / bt;
        const double mm = c + mp;
        const double aa = p.a0 + 0.5 * Nk;
        double bb = p.b0 + 0.5 * (T2q + p.beta0 * m0p * m0p - bt * mp * mp);
        if (bb < p.b0) bb = p.b0;
        nmv[it] = mm;
        nbt[it] = bt;
        nav[it] = aa;
        nbv[it] = bb;
        const double elt = sh.psi_a[k] - log(bb);
        const double tb = aa / bb;
        if (!init_mode) {
            double sq = T2q - 2.0 * mp * T1q + Nk * mp * mp;  // sum r (x - m)^2
            if (sq < 0.0) sq = 0.0;
            const double dm0 = mp - m0p;                        // m - m0
            acc += 0.5 * (Nk * (elt - kLn2Pi) - tb * sq - Nk / bt);
            acc += prior_const + 0.5 * elt - 0.5 * p.beta0 * (tb * dm0 * dm0 + 1.0 / bt) + (p.a0 - 1.0) * elt
                   - p.b0 * tb;
            acc -= 0.5 * sh.ln_bt[k] + 0.5 * elt - 0.5 + aa * log(bb) - sh.lg_a[k] + (aa - 1.0) * elt - aa;
        }
        sh.tmp[q] = coef_item(v, q, mm, bt, aa, bb, elt);
        if (!isfinite(mm) || !isfinite(bb) || !isfinite(elt) || !isfinite(T2q)) bad = 1;
    }
    if (bad) atomicOr(&sh.bad, 1);
    __syncthreads();
    coef_rows(v, sh, &p, !init_mode);
    {
        const double ws = wave_sum(acc);
        if ((tid & 63) == 0) sh.red[tid >> 6] = ws;
        __syncthreads();
        if (tid == 0)
            for (int w = 1; w < kMBlock / 64; ++w) sh.red[0] += sh.red[w];
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
            double L = sh.red[0] + total(v, K + 2 * KG);  // + H, the entropy of the responsibilities
            L += sh.lg_prior - sh.lg_asum;
            for (int k = 0; k < K; ++k) L += sh.term_k[k];
            if (!isfinite(L)) sh.bad = 1;
            if (sh.bad) {
                ctl->numeric = 1;
            } else {
                const int t = ctl->call_sweeps + 1;
                if (t >= 2 && fabs(L - ctl->elbo) <= ctl->tol * fabs(L)) ctl->converged = 1;
                ctl->elbo_prev = ctl->elbo;
                ctl->elbo = L;
                v.hist[(t - 1) % s.hist_cap] = L;
                ctl->call_sweeps = t;
                ctl->sweeps += 1;
            }
        }
    }
    __syncthreads();
    if (sh.bad) return;
    if (tid < K) v.alpha[tid] = v.nalpha[tid];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int q = tid + it * kMBlock;
        if (q >= KG) break;
        v.m[q] = nmv[it];
        v.beta[q] = nbt[it];
        v.a[q] = nav[it];
        v.b[q] = nbv[it];
    }
}

__global__ __launch_bounds__(kMBlock) void k_mstep(Shape s, Bufs bf, Prior p, int init_mode)
{
    __shared__ MShared sh;
    if (s.B == 1) {  // a single dataset: no work list
        mstep_one(s, bf, p, init_mode, 0, sh);
        return;
    }
    const int nds = n_active_datasets(s, bf);
    for (int slot = blockIdx.x; slot < nds; slot += gridDim.x) {
        mstep_one(s, bf, p, init_mode, bf.act_ds[slot], sh);
        __syncthreads();  // sh is rewritten by the next dataset
    }
}

hipError_t launch_reduce(const Shape &s, const Bufs &b, int init_mode, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce, dim3((s.Smax + 63) / 64, s.dgrid, red_split_max(s.Nmax)), dim3(kRedBlock), 0, st, s,
                       b, init_mode);
    return hipGetLastError();
}

hipError_t launch_mstep(const Shape &s, const Bufs &b, const Prior &p, int init_mode, hipStream_t st)
{
    hipLaunchKernelGGL(k_mstep, dim3(s.dgrid), dim3(kMBlock), 0, st, s, b, p, init_mode);
    return hipGetLastError();
}

hipError_t launch_coef(const Shape &s, const Bufs &b, hipStream_t st)
{
    hipLaunchKernelGGL(k_coef, dim3(s.B), dim3(kMBlock), 0, st, s, b);
    return hipGetLastError();
}

}  // namespace cavi
