// gfx950 kernels of the mixture CAVI sweep.
//
// One sweep (eq 12 applied to each factor of the mean-field family of eqs 9
// and 13, Section 3.4) is three launches:
//   k_estep_stats  expected log-likelihood of every row under every
//                  subpopulation, log-sum-exp responsibilities, and per-chunk
//                  sufficient statistics (weighted counts, sums and sums of
//                  squares around the previous mean, entropy);
//   k_reduce       fixed-order FP64 sum of the chunk partials;
//   k_mstep        conjugate updates (forms of eqs 16, 17, 24), the lower
//                  bound (eqs 10-11), the convergence test, and the FP32
//                  coefficients of the next E-step (expectations of eqs 26-31).
#include <math.h>

#include "cavi_impl.h"

namespace cavi {

namespace {

constexpr int kMaxItems = kMaxKG / kBlock;  // (k, g) items per thread

// Squared distance in FP64 with separate multiply and add (no contraction),
// so that the host reproduces it bit for bit.
__device__ __forceinline__ double sqdist64(const float *x, const float *y, int G)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int g = 0; g < G; ++g) {
        double d = (double)x[g] - (double)y[g];
        s = s + d * d;
    }
    return s;
}

template <int KT>
__device__ __forceinline__ void row_loglik(const float *xr, int G, int K, const float2 *__restrict__ hq,
                                           const float *__restrict__ cc, float (&l)[KT])
{
#pragma unroll
    for (int k = 0; k < KT; ++k) l[k] = 0.f;
    for (int g = 0; g < G; ++g) {
        const float xv = xr[g];
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            if (k < K) {
                const float2 c = hq[k * G + g];
                const float u = fmaf(xv, c.x, c.y);
                l[k] = fmaf(u, u, l[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KT; ++k)
        if (k < K) l[k] = cc[k] - l[k];
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// E-step + statistics.  Grid-stride over 2048-row chunks; each chunk is staged
// through LDS in tiles of tile_rows rows (row stride G+1 floats).  One thread
// owns one row for the E-step; for the statistics one thread owns (k, g) items
// and walks the tile's rows, skipping rows whose responsibility is exactly 0.
// init_mode: responsibilities are the hard nearest-seed assignment instead.
template <int KT>
__global__ __launch_bounds__(kBlock) void k_estep_stats(Shape s, const float *__restrict__ x,
                                                        const float *__restrict__ cc,
                                                        const float2 *__restrict__ hq,
                                                        const float *__restrict__ mf,
                                                        const float *__restrict__ seeds,
                                                        double *__restrict__ partials,
                                                        const Ctl *__restrict__ ctl, int init_mode)
{
    if (!init_mode && sweep_skipped(ctl)) return;
    extern __shared__ float smem[];
    __shared__ double red[kBlock];
    const int G = s.G, K = s.K, KG = K * G;
    const int TR = s.tile_rows, XS = G + 1, RS = KT + 1;
    float *xs = smem;
    float *rs = smem + TR * XS;
    const int tid = threadIdx.x;
    const int nit = (KG + kBlock - 1) / kBlock;

    float mfv[kMaxItems];
#pragma unroll
    for (int it = 0; it < kMaxItems; ++it) {
        const int p = tid + it * kBlock;
        mfv[it] = (it < nit && p < KG) ? mf[p] : 0.f;
    }

    for (int chunk = blockIdx.x; chunk < s.nchunk; chunk += gridDim.x) {
        double a1[kMaxItems], a2[kMaxItems];
#pragma unroll
        for (int it = 0; it < kMaxItems; ++it) a1[it] = a2[it] = 0.0;
        double t0 = 0.0, hh = 0.0;
        const int64_t r0 = (int64_t)chunk * kChunkRows;
        const int64_t r1 = min(s.N, r0 + kChunkRows);
        for (int64_t t = r0; t < r1; t += TR) {
            const int nr = (int)min((int64_t)TR, r1 - t);
            const float *src = x + t * G;
            const int tot = nr * G;
            for (int i = tid; i < tot; i += kBlock) {
                const int rr = i / G;
                xs[rr * XS + (i - rr * G)] = src[i];
            }
            __syncthreads();
            if (tid < TR) {
                float *rrow = rs + tid * RS;
                if (tid < nr) {
                    const float *xr = xs + tid * XS;
                    if (init_mode) {
                        int best = 0;
                        double bd = 0.0;
                        for (int j = 0; j < K; ++j) {
                            const double d2 = sqdist64(xr, seeds + j * G, G);
                            if (j == 0 || d2 < bd) {
                                bd = d2;
                                best = j;
                            }
                        }
#pragma unroll
                        for (int k = 0; k < KT; ++k) rrow[k] = (k == best) ? 1.f : 0.f;
                    } else {
                        float l[KT];
                        row_loglik<KT>(xr, G, K, hq, cc, l);
                        float mx = l[0];
#pragma unroll
                        for (int k = 1; k < KT; ++k)
                            if (k < K) mx = fmaxf(mx, l[k]);
                        float se = 0.f;
#pragma unroll
                        for (int k = 0; k < KT; ++k)
                            if (k < K) se += __expf(l[k] - mx);
                        const float L = mx + __logf(se);
                        // a non-finite row normaliser poisons the entropy so the update rejects the sweep
                        float h = isfinite(L) ? 0.f : __int_as_float(0x7fc00000);
#pragma unroll
                        for (int k = 0; k < KT; ++k) {
                            float v = 0.f;
                            if (k < K) {
                                const float dl = l[k] - L;
                                if (dl > -kLogRCut) {
                                    v = __expf(dl);
                                    h -= v * dl;
                                }
                            }
                            rrow[k] = v;
                        }
                        hh += (double)h;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < KT; ++k) rrow[k] = 0.f;
                }
            }
            __syncthreads();
#pragma unroll
            for (int it = 0; it < kMaxItems; ++it) {
                const int p = tid + it * kBlock;
                if (it < nit && p < KG) {
                    const int k = p / G, g = p - k * G;
                    const float c = mfv[it];
                    float s1 = 0.f, s2 = 0.f;
                    for (int j = 0; j < nr; ++j) {
                        const float rr = rs[j * RS + k];
                        if (rr != 0.f) {
                            const float d = xs[j * XS + g] - c;
                            const float w = rr * d;
                            s1 += w;
                            s2 = fmaf(w, d, s2);
                        }
                    }
                    a1[it] += (double)s1;
                    a2[it] += (double)s2;
                }
            }
            if (tid < K) {
                float s0 = 0.f;
                for (int j = 0; j < nr; ++j) s0 += rs[j * RS + tid];
                t0 += (double)s0;
            }
            __syncthreads();
        }
        red[tid] = hh;
        __syncthreads();
        for (int off = kBlock / 2; off > 0; off >>= 1) {
            if (tid < off) red[tid] += red[tid + off];
            __syncthreads();
        }
        double *out = partials + (size_t)chunk * s.S;
        if (tid < K) out[tid] = t0;
#pragma unroll
        for (int it = 0; it < kMaxItems; ++it) {
            const int p = tid + it * kBlock;
            if (it < nit && p < KG) {
                out[K + p] = a1[it];
                out[K + KG + p] = a2[it];
            }
        }
        if (tid == 0) out[K + 2 * KG] = red[0];
        __syncthreads();
    }
}

__global__ void k_ctl_begin(Ctl *ctl, int max_call, int stop_on_conv, double tol, int reset)
{
    ctl->max_call = max_call;
    ctl->stop_on_conv = stop_on_conv;
    ctl->tol = tol;
    ctl->call_sweeps = 0;
    ctl->converged = 0;
    ctl->numeric = 0;
    if (reset) {
        ctl->sweeps = 0;
        ctl->elbo = 0.0;
        ctl->elbo_prev = 0.0;
    }
}

// ---------------------------------------------------------------------------------------------
// Prior centre m0 = per-gene mean of X: per-chunk FP64 column sums, then a
// fixed-order sum over chunks.
__global__ __launch_bounds__(kBlock) void k_colpart(Shape s, const float *__restrict__ x, double *__restrict__ colpart)
{
    const int G = s.G;
    const int64_t r0 = (int64_t)blockIdx.x * kChunkRows, r1 = min(s.N, r0 + kChunkRows);
    for (int g = threadIdx.x; g < G; g += kBlock) {
        double acc = 0.0;
        for (int64_t r = r0; r < r1; ++r) acc += (double)x[r * G + g];
        colpart[(size_t)blockIdx.x * G + g] = acc;
    }
}

__global__ __launch_bounds__(kBlock) void k_colmean(Shape s, const double *__restrict__ colpart, double *__restrict__ m0)
{
    for (int g = threadIdx.x; g < s.G; g += kBlock) {
        double acc = 0.0;
        for (int c = 0; c < s.nchunk; ++c) acc += colpart[(size_t)c * s.G + g];
        m0[g] = acc / (double)s.N;
    }
}

// ---------------------------------------------------------------------------------------------
// k-means++ helpers: running minimum of the squared distance to the seeds
// chosen so far, its per-block maximum, and per-block sums of the integer
// weights floor(minD2 * 2^e).
__global__ __launch_bounds__(kBlock) void k_d2(Shape s, const float *__restrict__ x, const float *__restrict__ seed,
                                               double *__restrict__ mind2, double *__restrict__ blockmax, int first)
{
    __shared__ double red[kBlock];
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v = 0.0;
    if (n < s.N) {
        const double d2 = sqdist64(x + n * s.G, seed, s.G);
        v = first ? d2 : fmin(mind2[n], d2);
        mind2[n] = v;
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) blockmax[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_wsum(Shape s, const double *__restrict__ mind2, int e,
                                                 unsigned long long *__restrict__ blocksum)
{
    __shared__ unsigned long long red[kBlock];
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long w = 0;
    if (n < s.N) w = (unsigned long long)floor(ldexp(mind2[n], e));
    red[threadIdx.x] = w;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) blocksum[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------------------------
// Responsibilities of the current coefficients, one thread per row.
template <int KT>
__global__ __launch_bounds__(kBlock) void k_resp(Shape s, const float *__restrict__ x, const float *__restrict__ cc,
                                                 const float2 *__restrict__ hq, float *__restrict__ r)
{
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= s.N) return;
    const int K = s.K;
    float l[KT];
    row_loglik<KT>(x + n * s.G, s.G, K, hq, cc, l);
    float mx = l[0];
#pragma unroll
    for (int k = 1; k < KT; ++k)
        if (k < K) mx = fmaxf(mx, l[k]);
    float se = 0.f;
#pragma unroll
    for (int k = 0; k < KT; ++k)
        if (k < K) se += __expf(l[k] - mx);
    const float L = mx + __logf(se);
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        if (k < K) {
            const float dl = l[k] - L;
            r[n * K + k] = dl > -kLogRCut ? __expf(dl) : 0.f;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// host-side helpers and launchers

int choose_kt(int K)
{
    return K <= 4 ? 4 : K <= 8 ? 8 : K <= 16 ? 16 : K <= 32 ? 32 : 64;
}

int choose_tile_rows(int G, int kt)
{
    const size_t per_row = (size_t)(G + 1 + kt + 1) * sizeof(float);
    // dynamic LDS budget: the device's per-block limit less the static arrays
    const size_t budget = (size_t)(g_lds_limit > 0 ? g_lds_limit : 65536) - 4096;
    int tr = 256;
    while (tr > 16 && (size_t)tr * per_row > budget) tr -= 16;
    return (size_t)tr * per_row > budget ? 0 : tr;
}

static size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

size_t workspace_bytes(const Shape &s)
{
    const size_t K = s.K, KG = (size_t)s.K * s.G, G = s.G;
    size_t n = 0;
    n += 2 * al(K * 8);                // alpha, nalpha
    n += 9 * al(KG * 8);               // m beta a b, nm nbeta na nb, tmp
    n += al(G * 8);                    // m0
    n += al(K * 4) + al(2 * KG * 4) + 2 * al(KG * 4);  // cc, hq, mf, seeds
    n += al((size_t)s.nchunk * s.S * 8);
    n += al((size_t)s.S * 8);
    n += al((size_t)kHist * 8);
    n += al(sizeof(Ctl));
    n += al((size_t)s.N * 8);
    n += al((size_t)s.nblk * 8) * 2;
    n += al((size_t)s.nchunk * G * 8);
    return n;
}

void carve(const Shape &s, void *ws, Bufs &b)
{
    const size_t K = s.K, KG = (size_t)s.K * s.G, G = s.G;
    char *p = (char *)ws;
    auto take = [&](size_t bytes) {
        void *r = p;
        p += al(bytes);
        return r;
    };
    b.alpha = (double *)take(K * 8);
    b.nalpha = (double *)take(K * 8);
    b.m = (double *)take(KG * 8);
    b.beta = (double *)take(KG * 8);
    b.a = (double *)take(KG * 8);
    b.b = (double *)take(KG * 8);
    b.nm = (double *)take(KG * 8);
    b.nbeta = (double *)take(KG * 8);
    b.na = (double *)take(KG * 8);
    b.nb = (double *)take(KG * 8);
    b.tmp = (double *)take(KG * 8);
    b.m0 = (double *)take(G * 8);
    b.cc = (float *)take(K * 4);
    b.hq = (float *)take(2 * KG * 4);
    b.mf = (float *)take(KG * 4);
    b.seeds = (float *)take(KG * 4);
    b.partials = (double *)take((size_t)s.nchunk * s.S * 8);
    b.totals = (double *)take((size_t)s.S * 8);
    b.hist = (double *)take((size_t)kHist * 8);
    b.ctl = (Ctl *)take(sizeof(Ctl));
    b.mind2 = (double *)take((size_t)s.N * 8);
    b.blockmax = (double *)take((size_t)s.nblk * 8);
    b.blocksum = (unsigned long long *)take((size_t)s.nblk * 8);
    b.colpart = (double *)take((size_t)s.nchunk * G * 8);
}

template <int KT>
static hipError_t launch_estep_t(const Shape &s, const Bufs &b, int init_mode, hipStream_t st)
{
    const size_t lds = (size_t)s.tile_rows * (s.G + 1 + KT + 1) * sizeof(float);
    hipLaunchKernelGGL(k_estep_stats<KT>, dim3(s.nchunk), dim3(kBlock), lds, st, s, b.x, b.cc,
                       (const float2 *)b.hq, b.mf, b.seeds, b.partials, b.ctl, init_mode);
    return hipGetLastError();
}

hipError_t prepare_kernels()
{
    static bool done = false;
    if (done) return hipSuccess;
    int dev = 0, per_block = 0, optin = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    (void)hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    (void)hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev);
    (void)hipGetLastError();
    g_lds_limit = per_block > optin ? per_block : optin;
    // Raising the dynamic limit is only needed (and only accepted) where the
    // opt-in limit exceeds the default one; failures here are not fatal, the
    // tile size below is chosen against the limit that the device reports.
    if (optin > per_block) {
        const int want = optin - 4096;
        (void)hipFuncSetAttribute((const void *)k_estep_stats<4>, hipFuncAttributeMaxDynamicSharedMemorySize, want);
        (void)hipFuncSetAttribute((const void *)k_estep_stats<8>, hipFuncAttributeMaxDynamicSharedMemorySize, want);
        (void)hipFuncSetAttribute((const void *)k_estep_stats<16>, hipFuncAttributeMaxDynamicSharedMemorySize, want);
        (void)hipFuncSetAttribute((const void *)k_estep_stats<32>, hipFuncAttributeMaxDynamicSharedMemorySize, want);
        (void)hipFuncSetAttribute((const void *)k_estep_stats<64>, hipFuncAttributeMaxDynamicSharedMemorySize, want);
        (void)hipGetLastError();
    }
    done = true;
    return hipSuccess;
}

int g_lds_limit = 0;

hipError_t launch_estep_stats(const Shape &s, const Bufs &b, int init_mode, hipStream_t st)
{
    if (!init_mode && tiled_supported(s.K, s.G)) return launch_estep_tiled(s, b, st);
    switch (s.kt) {
    case 4: return launch_estep_t<4>(s, b, init_mode, st);
    case 8: return launch_estep_t<8>(s, b, init_mode, st);
    case 16: return launch_estep_t<16>(s, b, init_mode, st);
    case 32: return launch_estep_t<32>(s, b, init_mode, st);
    default: return launch_estep_t<64>(s, b, init_mode, st);
    }
}




hipError_t launch_prior_mean(const Shape &s, const Bufs &b, hipStream_t st)
{
    hipLaunchKernelGGL(k_colpart, dim3(s.nchunk), dim3(kBlock), 0, st, s, b.x, b.colpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colmean, dim3(1), dim3(kBlock), 0, st, s, b.colpart, b.m0);
    return hipGetLastError();
}

hipError_t launch_d2(const Shape &s, const Bufs &b, int seed_index, int first, hipStream_t st)
{
    hipLaunchKernelGGL(k_d2, dim3(s.nblk), dim3(kBlock), 0, st, s, b.x, b.seeds + (size_t)seed_index * s.G, b.mind2,
                       b.blockmax, first);
    return hipGetLastError();
}

hipError_t launch_wsum(const Shape &s, const Bufs &b, int e, hipStream_t st)
{
    hipLaunchKernelGGL(k_wsum, dim3(s.nblk), dim3(kBlock), 0, st, s, b.mind2, e, b.blocksum);
    return hipGetLastError();
}

hipError_t launch_resp(const Shape &s, const Bufs &b, float *r, hipStream_t st)
{
    const dim3 grid(s.nblk);
    switch (s.kt) {
    case 4: hipLaunchKernelGGL(k_resp<4>, grid, dim3(kBlock), 0, st, s, b.x, b.cc, (const float2 *)b.hq, r); break;
    case 8: hipLaunchKernelGGL(k_resp<8>, grid, dim3(kBlock), 0, st, s, b.x, b.cc, (const float2 *)b.hq, r); break;
    case 16: hipLaunchKernelGGL(k_resp<16>, grid, dim3(kBlock), 0, st, s, b.x, b.cc, (const float2 *)b.hq, r); break;
    case 32: hipLaunchKernelGGL(k_resp<32>, grid, dim3(kBlock), 0, st, s, b.x, b.cc, (const float2 *)b.hq, r); break;
    default: hipLaunchKernelGGL(k_resp<64>, grid, dim3(kBlock), 0, st, s, b.x, b.cc, (const float2 *)b.hq, r); break;
    }
    return hipGetLastError();
}

hipError_t launch_ctl_begin(const Bufs &b, int max_call, int stop_on_conv, double tol, int reset, hipStream_t st)
{
    hipLaunchKernelGGL(k_ctl_begin, dim3(1), dim3(1), 0, st, b.ctl, max_call, stop_on_conv, tol, reset);
    return hipGetLastError();
}

}  // namespace cavi
