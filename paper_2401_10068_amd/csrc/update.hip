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
constexpr int kRedBlock = 1024;  // k_reduce: 16 waves per 64 statistics (a single dataset)
constexpr int kRedBatchBlock = 256;  // k_reduce for batches: 4 waves running the 16 wave slots
constexpr int kRedBatchGrid = 2048;  // datasets a batch's reduction takes at once
constexpr int kMBlock = 1024;    // k_mstep (one dataset), k_coef: one (k, g) item per thread up to K G = 1024
constexpr int kMBatchBlock = 256;  // k_mstep_batch: a batch's datasets are small; 256 threads leave
                                   // the update its registers and fit three workgroups per CU
constexpr int kMBatchGrid = 2048;  // datasets a batch's update takes at once

// Sum over the 64 lanes of a wave with a fixed butterfly (same order every run).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NT>
struct MShared {
    double red[kMaxKG / 64];  // the bound's item terms, one sum per group of 64 items (see mstep_one)
    double ak[kMaxK], psi_ak[kMaxK], lg_ak[kMaxK], term_k[kMaxK];
    double psi_a[kMaxK], lg_a[kMaxK], ln_bt[kMaxK];  // per component: digamma, lgamma of a_kg; ln(beta_kg / 2 pi)
    double tmp[kMaxKG];
    double psum, lg_asum;                 // digamma, lgamma of sum(alpha)
    double lg_ka0, lg_alpha0, lg_a0;      // lgamma of K alpha0, alpha0, a0
    double ln_b0pi, ln_b0;                // ln(beta0 / 2 pi), ln b0
    int bad;
};

// Per-dataset views of the batch arrays.
struct View {
    int K, G;
    double *alpha, *m, *beta, *a, *b;
    double *nm, *nbeta, *na, *nb;
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
    const Ds d = dataset(s, bf, bi);
    v.K = d.K;
    v.G = s.G;
    v.alpha = bf.alpha + kb;
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
    v.nsplit = red_split(d.nchunk);
    v.hist = bf.hist + (size_t)bi * s.hist_cap;
    v.ctl = bf.ctl + bi;
    return v;
}

// Statistic i of the dataset: the sums of its chunk ranges, added in range order.  The
// kRedSplit loads are issued without a branch (a dataset of one range reads its single sum
// kRedSplit times), so that the loads of several statistics can be in flight together.
struct Tot {
    double r[kRedSplit];
};

__device__ __forceinline__ Tot load_total(const View &v, int i)
{
    const double *t = v.totals + i;
    const size_t stride = v.nsplit > 1 ? v.smax : 0;
    Tot o;
#pragma unroll
    for (int z = 0; z < kRedSplit; ++z) o.r[z] = t[z * stride];
    return o;
}

__device__ __forceinline__ double sum_total(const View &v, const Tot &o)
{
    double sum = o.r[0];
#pragma unroll
    for (int z = 1; z < kRedSplit; ++z) sum += o.r[z];
    return v.nsplit > 1 ? sum : o.r[0];
}

__device__ __forceinline__ double total(const View &v, int i) { return sum_total(v, load_total(v, i)); }

// Per-(k,g) coefficients of the E-step from one subpopulation-gene state:
//   l_nk = c_k - sum_g (h x + q)^2,  h = sqrt(E[tau]/2),  q = -m h,
//   c_k  = E ln pi_k + sum_g tmp_kg,  tmp = (E ln tau - ln 2pi - 1/beta) / 2.
__device__ __forceinline__ void coef_hq(const View &v, int q, double mm, double aa, double bb)
{
    const float hf = (float)sqrt(0.5 * aa / bb);
    v.hq[2 * q] = hf;
    v.hq[2 * q + 1] = (float)(-mm * (double)hf);
    v.mf[q] = (float)mm;
}

__device__ __forceinline__ double coef_item(const View &v, int q, double mm, double bt, double aa, double bb,
                                            double elt)
{
    coef_hq(v, q, mm, aa, bb);
    return 0.5 * (elt - kLn2Pi - 1.0 / bt);
}

// c_k from the per-(k,g) parts in LDS: wave w sums subpopulations w, w+16, ...
template <int NT>
__device__ __forceinline__ void coef_rows(const View &v, MShared<NT> &sh)
{
    const int G = v.G, K = v.K;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = wv; k < K; k += NT / 64) {
        double x = 0.0;
        for (int g = lane; g < G; g += 64) x += sh.tmp[k * G + g];
        x = wave_sum(x);
        if (lane == 0) {
            const double elnpi = sh.psi_ak[k] - sh.psum;
            const double c = elnpi + x;
            v.cc[k] = (float)c;
            if (!isfinite(c)) sh.bad = 1;
        }
    }
}

}  // namespace

// totals[b][z][i] = sum over the chunks of range z of dataset b (its chunks [z n / Z, (z + 1) n / Z)
// for Z = red_split(n)) of partials[chunk][i], in a fixed order: wave v of the block sums a
// contiguous 1/16 of the range's chunks (4 interleaved accumulators), then the 16 wave sums are added
// in wave order.  The ranges spread a large dataset over Z workgroups per 64 statistics; the update
// adds them.
// The sixteen wave slots of the order above are taken by NT / 64 waves, each running 1024 / NT
// slots in turn (one for a single dataset's 1024-thread blocks; four for a batch's 256-thread
// blocks, whose datasets are mostly a few chunks each), so both give the same sums.
template <int NT>
__global__ __launch_bounds__(NT) void k_reduce(Shape s, Bufs bf, int init_mode)
{
    constexpr int nw = kRedBlock / 64;    // wave slots of the summation order
    constexpr int per = nw / (NT / 64);   // slots per wave
    __shared__ double part[nw][64];
    const int lane = threadIdx.x & 63, rw = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int z = blockIdx.z;
    const int nds = n_active_datasets(s, bf);
    for (int slot = blockIdx.y; slot < nds; slot += gridDim.y) {
        const int bi = active_dataset(s, bf, slot);
        const Ds d = dataset(s, bf, bi);
        const int S = d.K + 2 * d.K * s.G + 1;
        if (blockIdx.x * 64 >= S) continue;
        const int Z = red_split(d.nchunk);
        if (z >= Z) continue;
        // 32-bit products: a dataset has fewer than 2^31 rows, so fewer than 2^20 chunks
        const int r0 = (d.nchunk * z) / Z, r1 = (d.nchunk * (z + 1)) / Z;
        const int nr = r1 - r0;
        // lanes past the statistics read the last one (their sums are not stored)
        const double *base = bf.partials + (size_t)(d.chunk0 + r0) * s.Smax + min(i, S - 1);
        // a slot's chunks in batches of eight loads in flight (indices clamped to the slot's last
        // chunk); the first batch of the wave's first slot is requested before the skip test
        double L[8];
        auto load8 = [&](const double *pp, int n, int b0) {
#pragma unroll
            for (int k = 0; k < 8; ++k) L[k] = pp[(size_t)min(b0 + k, n - 1) * s.Smax];
        };
        int c0 = (nr * (rw * per)) / nw, n = (nr * (rw * per + 1)) / nw - c0;
        if (n > 0) load8(base + (size_t)c0 * s.Smax, n, 0);
        if (!init_mode && sweep_skipped(bf.ctl + bi)) continue;
        for (int u = 0; u < per; ++u) {
            const int wv = rw * per + u;  // the slot
            if (u > 0) {
                c0 = (nr * wv) / nw;
                n = (nr * (wv + 1)) / nw - c0;
                if (n > 0) load8(base + (size_t)c0 * s.Smax, n, 0);
            }
            const int n4 = n & ~3;  // the slot's chunks in whole groups of four
            const double *pp = base + (size_t)c0 * s.Smax;
            double q[4] = {0.0, 0.0, 0.0, 0.0};
            for (int b0 = 0; b0 < n; b0 += 8) {
                if (b0 > 0) load8(pp, n, b0);
                // chunk t adds to accumulator t mod 4 while in a whole group of four, else to the first
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int t = b0 + k;
                    if (t < n4) q[k & 3] += L[k];
                    else if (t < n) q[0] += L[k];
                }
            }
            part[wv][lane] = (q[0] + q[1]) + (q[2] + q[3]);
        }
        __syncthreads();
        if (rw == 0 && i < S) {
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
    __shared__ MShared<kMBlock> sh;
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
    coef_rows(v, sh);
}

// Conjugate updates from the totals, written with sums around the E-step's
// FP32 centre c = mf:  T1 = sum r (x - c),  T2 = sum r (x - c)^2,
//   alpha = alpha0 + N_k;  beta = beta0 + N_k;  m = c + (beta0 (m0 - c) + T1) / beta;
//   a = a0 + N_k / 2;  b = b0 + [T2 + beta0 (m0 - c)^2 - beta (m - c)^2] / 2,
// then the lower bound at the new q(pi), q(mu, tau) with the entropy H of the
// responsibilities.  A non-finite value leaves the state untouched and raises
// ctl->numeric.
template <int NT>
__device__ __forceinline__ void mstep_one(const Shape &s, const Bufs &bf, const Prior &p, int init_mode, int bi,
                                          MShared<NT> &sh)
{
    const View v = view(s, bf, bi);
    Ctl *ctl = v.ctl;
    const int G = v.G, K = v.K, KG = K * G, tid = threadIdx.x;
    const int lane = tid & 63, role = NT / 64 - 1 - (tid >> 6);  // roles from the last wave down
    // Every statistic this thread reads is requested at once, before the skip test, so that one
    // memory latency covers them all: its first item (q = tid; clamped indices where the thread
    // has none), the count of its lane's subpopulation, the entropy.
    const int q0 = tid, k0 = q0 / G;
    const bool has0 = q0 < KG;
    const int qc = has0 ? q0 : KG - 1, kc = qc / G;
    const Tot lN = load_total(v, kc), lT1 = load_total(v, K + qc), lT2 = load_total(v, K + KG + qc);
    const Tot lR = load_total(v, lane < K ? lane : 0), lH = load_total(v, K + 2 * KG);
    const float c0 = v.mf[qc];
    const double m00 = v.m0[qc - kc * G];
    // the control-block fields thread 0 updates at the end (only it writes them), read now as well
    const int cs0 = ctl->call_sweeps, sw0 = ctl->sweeps;
    const double elbo0 = ctl->elbo, tol0 = ctl->tol;
    if (!init_mode && sweep_skipped(ctl)) return;
    const double N0 = sum_total(v, lN), T10 = sum_total(v, lT1), T20 = sum_total(v, lT2);
    const double nr = sum_total(v, lR), Hq = sum_total(v, lH);
    if (tid == 0) sh.bad = 0;

    // Special functions, one function per wave and one argument per lane, in the last three waves
    // (which hold no items while K G <= NT - 192), while the item threads run the parts of their
    // updates that do not need them.  Digamma (last wave) and lgamma (the one before) of
    // alpha_k = alpha0 + N_k, of a_kg = a0 + N_k / 2 (the same for every gene of a subpopulation) and
    // of sum(alpha); the lgamma wave adds K alpha0, alpha0 and a0.  Logarithms (third from last) of
    // beta_kg / 2 pi, beta0 / 2 pi and b0.  Lane k holds N_k.
    if (role == 0 || (!init_mode && role <= 2)) {
        const double asum = wave_sum(lane < K ? p.alpha0 + nr : 0.0);
        const int nslot = role == 0 ? 2 * K + 1 : (role == 1 ? 2 * K + 4 : K + 2);
        for (int j0 = 0; j0 < nslot; j0 += 64) {
            const int j = j0 + lane;
            const double nk = __shfl(nr, j < K ? j : (j < 2 * K ? j - K : 0), 64);
            if (j >= nslot) continue;
            if (role == 2) {
                const double y = log(j < K ? (p.beta0 + nk) / kTwoPi : (j == K ? p.beta0 / kTwoPi : p.b0));
                if (j < K) sh.ln_bt[j] = y;
                else if (j == K) sh.ln_b0pi = y;
                else sh.ln_b0 = y;
                continue;
            }
            double x = j < K ? p.alpha0 + nk : (j < 2 * K ? p.a0 + 0.5 * nk : asum);
            if (j > 2 * K) x = j == 2 * K + 1 ? K * p.alpha0 : (j == 2 * K + 2 ? p.alpha0 : p.a0);
            if (role == 0) {
                const double y = dev_digamma(x);
                if (j < K) {
                    sh.ak[j] = x;
                    sh.psi_ak[j] = y;
                } else if (j < 2 * K) {
                    sh.psi_a[j - K] = y;
                } else {
                    sh.psum = y;
                }
            } else {
                const double y = dev_lgamma(x);
                if (j < K) sh.lg_ak[j] = y;
                else if (j < 2 * K) sh.lg_a[j - K] = y;
                else if (j == 2 * K) sh.lg_asum = y;
                else if (j == 2 * K + 1) sh.lg_ka0 = y;
                else if (j == 2 * K + 2) sh.lg_alpha0 = y;
                else sh.lg_a0 = y;
            }
        }
    }

    // first item, before the barrier: the update and everything of its bound term but E ln tau;
    // its new state stays in registers until the commit
    double nmv = 0.0, nbt = 0.0, nav = 0.0, nbv = 0.0;
    double lbb = 0.0, tb = 0.0, ibt = 0.0, nkbt = 0.0, sq = 0.0, dm0 = 0.0;
    bool fin0 = true;
    if (has0) {
        const double c = (double)c0;
        const double m0p = m00 - c;
        const double bt = p.beta0 + N0;
        const double mp = (p.beta0 * m0p + T10) / bt;
        const double mm = c + mp;
        const double aa = p.a0 + 0.5 * N0;
        double bb = p.b0 + 0.5 * (T20 + p.beta0 * m0p * m0p - bt * mp * mp);
        if (bb < p.b0) bb = p.b0;
        nmv = mm;
        nbt = bt;
        nav = aa;
        nbv = bb;
        lbb = log(bb);
        ibt = 1.0 / bt;
        if (!init_mode) {
            tb = aa / bb;
            nkbt = N0 / bt;
            sq = T20 - 2.0 * mp * T10 + N0 * mp * mp;  // sum r (x - m)^2
            if (sq < 0.0) sq = 0.0;
            dm0 = mp - m0p;                            // m - m0
        }
        coef_hq(v, q0, mm, aa, bb);
        fin0 = isfinite(mm) && isfinite(bb) && isfinite(T20);
    }
    __syncthreads();

    const double prior_const = init_mode ? 0.0 : 0.5 * sh.ln_b0pi + p.a0 * sh.ln_b0 - sh.lg_a0;
    double acc = 0.0;
    int bad = !fin0;
    if (has0) {
        const double elt = sh.psi_a[k0] - lbb;
        if (!isfinite(elt)) bad = 1;
        if (!init_mode) {
            const double aa = nav;
            acc += 0.5 * (N0 * (elt - kLn2Pi) - tb * sq - nkbt);
            acc += prior_const + 0.5 * elt - 0.5 * p.beta0 * (tb * dm0 * dm0 + ibt) + (p.a0 - 1.0) * elt - p.b0 * tb;
            acc -= 0.5 * sh.ln_bt[k0] + 0.5 * elt - 0.5 + aa * lbb - sh.lg_a[k0] + (aa - 1.0) * elt - aa;
        }
        sh.tmp[q0] = 0.5 * (elt - kLn2Pi - ibt);
    }
    // The bound's item terms are summed per group of 64 consecutive items (a wave sum each), and
    // the groups in item order, so that the sum does not depend on the block size: a dataset in a
    // batch (512-thread blocks) gets the bits of a single handle (1024).
    if (!init_mode) {
        const double ws = wave_sum(acc);
        if (lane == 0) sh.red[tid >> 6] = ws;
    }
    // further items (K G > NT), after the barrier; their new state is staged in nm, nbeta, na, nb
    for (int base = NT; base < KG; base += NT) {
        const int q = base + tid;
        double accq = 0.0;
        if (q < KG) {
            const int k = q / G, g = q - k * G;
            const double Nk = total(v, k);
            const double T1q = total(v, K + q), T2q = total(v, K + KG + q);
            const double c = (double)v.mf[q];
            const double m0p = v.m0[g] - c;
            const double bt = p.beta0 + Nk;
            const double mp = (p.beta0 * m0p + T1q) / bt;
            const double mm = c + mp;
            const double aa = p.a0 + 0.5 * Nk;
            double bb = p.b0 + 0.5 * (T2q + p.beta0 * m0p * m0p - bt * mp * mp);
            if (bb < p.b0) bb = p.b0;
            v.nm[q] = mm;
            v.nbeta[q] = bt;
            v.na[q] = aa;
            v.nb[q] = bb;
            const double elt = sh.psi_a[k] - log(bb);
            const double tbq = aa / bb;
            if (!init_mode) {
                double sqq = T2q - 2.0 * mp * T1q + Nk * mp * mp;
                if (sqq < 0.0) sqq = 0.0;
                const double dmq = mp - m0p;
                accq += 0.5 * (Nk * (elt - kLn2Pi) - tbq * sqq - Nk / bt);
                accq += prior_const + 0.5 * elt - 0.5 * p.beta0 * (tbq * dmq * dmq + 1.0 / bt) + (p.a0 - 1.0) * elt
                        - p.b0 * tbq;
                accq -= 0.5 * sh.ln_bt[k] + 0.5 * elt - 0.5 + aa * log(bb) - sh.lg_a[k] + (aa - 1.0) * elt - aa;
            }
            sh.tmp[q] = coef_item(v, q, mm, bt, aa, bb, elt);
            if (!isfinite(mm) || !isfinite(bb) || !isfinite(elt) || !isfinite(T2q)) bad = 1;
        }
        if (!init_mode) {
            const double ws = wave_sum(accq);
            if (lane == 0 && base + (tid & ~63) < KG) sh.red[q >> 6] = ws;
        }
    }
    if (bad) atomicOr(&sh.bad, 1);
    if (!init_mode && role == 0 && lane < K) {  // the q(pi) terms of the bound
        const double ak = sh.ak[lane], elnpi = sh.psi_ak[lane] - sh.psum;
        sh.term_k[lane] = nr * elnpi + (p.alpha0 - 1.0) * elnpi + sh.lg_ak[lane] - (ak - 1.0) * elnpi;
    }
    __syncthreads();

    // c_k in every wave; the bound in thread 0 beside them
    coef_rows(v, sh);
    double L = 0.0;
    if (tid == 0 && !init_mode) {
        double r = sh.red[0];
        for (int w = 1; w < (KG + 63) / 64; ++w) r += sh.red[w];
        L = r + Hq;  // + H, the entropy of the responsibilities
        const double lg_prior = sh.lg_ka0 - K * sh.lg_alpha0;
        L += lg_prior - sh.lg_asum;
        for (int k = 0; k < K; ++k) L += sh.term_k[k];
        if (!isfinite(L)) sh.bad = 1;
    }
    __syncthreads();
    const bool failed = sh.bad != 0;
    if (tid == 0) {
        if (init_mode) {
            if (!failed) {
                ctl->sweeps = 0;
                ctl->call_sweeps = 0;
                ctl->converged = 0;
                ctl->numeric = 0;
                ctl->elbo = 0.0;
            } else {
                ctl->numeric = 1;
            }
        } else if (failed) {
            ctl->numeric = 1;
        } else {
            const int t = cs0 + 1;
            if (t >= 2 && fabs(L - elbo0) <= tol0 * fabs(L)) ctl->converged = 1;
            ctl->elbo_prev = elbo0;
            ctl->elbo = L;
            v.hist[(t - 1) % s.hist_cap] = L;
            ctl->call_sweeps = t;
            ctl->sweeps = sw0 + 1;
        }
    }
    if (failed) return;
    if (tid < K) v.alpha[tid] = sh.ak[tid];
    if (has0) {
        v.m[q0] = nmv;
        v.beta[q0] = nbt;
        v.a[q0] = nav;
        v.b[q0] = nbv;
    }
    for (int q = tid + NT; q < KG; q += NT) {
        v.m[q] = v.nm[q];
        v.beta[q] = v.nbeta[q];
        v.a[q] = v.na[q];
        v.b[q] = v.nb[q];
    }
}

// a single dataset
__global__ __launch_bounds__(kMBlock) void k_mstep(Shape s, Bufs bf, Prior p, int init_mode)
{
    __shared__ MShared<kMBlock> sh;
    mstep_one<kMBlock>(s, bf, p, init_mode, 0, sh);
}

// a batch: the workgroups loop over the datasets on the work list
__global__ __launch_bounds__(kMBatchBlock) void k_mstep_batch(Shape s, Bufs bf, Prior p, int init_mode)
{
    __shared__ MShared<kMBatchBlock> sh;
    const int nds = n_active_datasets(s, bf);
    for (int slot = blockIdx.x; slot < nds; slot += gridDim.x) {
        mstep_one<kMBatchBlock>(s, bf, p, init_mode, bf.act_ds[slot], sh);
        __syncthreads();  // sh is rewritten by the next dataset
    }
}

hipError_t launch_reduce(const Shape &s, const Bufs &b, int init_mode, hipStream_t st)
{
    const dim3 grid((s.Smax + 63) / 64, s.B == 1 ? 1 : std::min(s.B, kRedBatchGrid), red_split_max(s.Nmax));
    if (s.B == 1)
        hipLaunchKernelGGL(k_reduce<kRedBlock>, grid, dim3(kRedBlock), 0, st, s, b, init_mode);
    else
        hipLaunchKernelGGL(k_reduce<kRedBatchBlock>, grid, dim3(kRedBatchBlock), 0, st, s, b, init_mode);
    return hipGetLastError();
}

hipError_t launch_mstep(const Shape &s, const Bufs &b, const Prior &p, int init_mode, hipStream_t st)
{
    if (s.B == 1)
        hipLaunchKernelGGL(k_mstep, dim3(1), dim3(kMBlock), 0, st, s, b, p, init_mode);
    else
        hipLaunchKernelGGL(k_mstep_batch, dim3(std::min(s.B, kMBatchGrid)), dim3(kMBatchBlock), 0, st, s, b, p,
                           init_mode);
    return hipGetLastError();
}

hipError_t launch_coef(const Shape &s, const Bufs &b, hipStream_t st)
{
    hipLaunchKernelGGL(k_coef, dim3(s.B), dim3(kMBlock), 0, st, s, b);
    return hipGetLastError();
}

}  // namespace cavi
