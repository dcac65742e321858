// Learned warm start of the batched CAVI path: per-dataset features, the
// training targets, a small MLP (hidden layers with GELU) trained and
// evaluated with BF16 MFMA products accumulated in FP32, and the conversion of
// its outputs into an initial variational state.
//
// Features of a dataset, per gene g (18 values, gene-major, 18 G in all):
//   (mean_g - 25) / 10, ln max(var_g, 1e-30) (population variance over all N rows), and
//   (c_gj - 25) / 10 for 16 rank-bin means c_gj: the first M = min(N, 4096) rows are
//   ranked by their row sum over genes (left-to-right FP64 sum; ties by row index), rank
//   bin j holds ranks [floor(j M / 16), max(floor((j+1) M / 16), floor(j M / 16) + 1)),
//   and c_gj is the mean of gene g over the rows of bin j (FP64, summed in rank order).
// Quantile features (k_features_q): the same moments, then (q_gj - 25) / 10 for the 16
// nearest-rank quantiles q_gj = sorted(x_g)[floor((j + 0.5) N / 16)] over all N rows.
// Targets of a generated dataset (K components sorted by their mean over
// genes, ascending, ties by index): (mu - 25) / 10 [K G], ln tau [K G], ln pi [K].
#include <math.h>

#include "cavi_impl.h"

namespace cavi {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kSortMax = 4096;  // rows ranked for the rank-bin features
constexpr int kTM = 64, kTN = 64, kTK = 32;  // GEMM tile

__device__ __forceinline__ __bf16 to_bf16(float f)
{
    // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    const unsigned short h = (unsigned short)(u >> 16);
    return __builtin_bit_cast(__bf16, h);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z)
{
    const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * __expf(-0.5f * z * z);
    return cdf + z * pdf;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// features: one workgroup per dataset
// ---------------------------------------------------------------------------------------------
// features: one workgroup per dataset
// slots 0 and 1 of every gene: (mean - 25) / 10 and ln max(var, 1e-30) over all N >= 1 rows
__device__ void feature_moments(const float *__restrict__ xd, int64_t N, int G, float *__restrict__ f)
{
    __shared__ double part[2 * kBlock];
    __shared__ double gmean[kMaxG];
    const int tid = threadIdx.x;
    // moments over all rows: lane slots (gene, row phase), RP rows per pass, coalesced along rows
    const int RP = G >= kBlock ? 1 : kBlock / G;
    for (int pass = 0; pass < 2; ++pass) {
        for (int g0 = 0; g0 < G; g0 += kBlock) {
            const int slots = G >= kBlock ? min(kBlock, G - g0) : RP * G;
            double s = 0.0;
            if (tid < slots) {
                const int g = G >= kBlock ? g0 + tid : tid % G;
                const int rp = G >= kBlock ? 0 : tid / G;
                const double mu = pass ? gmean[g] : 0.0;
                for (int64_t n = rp; n < N; n += RP) {
                    const double v = (double)xd[n * G + g];
                    s += pass ? (v - mu) * (v - mu) : v;
                }
            }
            part[tid] = s;
            __syncthreads();
            const int ng = G >= kBlock ? slots : G;
            for (int q = tid; q < ng; q += kBlock) {
                double t = 0.0;
                for (int r = 0; r < (G >= kBlock ? 1 : RP); ++r) t += part[r * G + q];
                const int g = (G >= kBlock ? g0 : 0) + q;
                if (pass == 0) {
                    gmean[g] = t / (double)N;
                    f[(size_t)g * 18] = (float)((t / (double)N - 25.0) / 10.0);
                } else {
                    f[(size_t)g * 18 + 1] = (float)log(fmax(t / (double)N, 1e-30));
                }
            }
            __syncthreads();
            if (G < kBlock) break;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_features(const float *__restrict__ x, const int64_t *__restrict__ row_off,
                                                     int G, float *__restrict__ feat)
{
    __shared__ double key[kSortMax];
    __shared__ int32_t rid[kSortMax];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int64_t r0 = row_off[b], N = row_off[b + 1] - r0;
    const float *xd = x + r0 * G;
    float *f = feat + (size_t)b * 18 * G;
    if (N <= 0) {  // empty dataset: no features (NaN)
        for (int q = tid; q < 18 * G; q += kBlock) f[q] = NAN;
        return;
    }
    feature_moments(xd, N, G, f);
    // rank the first M rows by their row sum (bitonic sort of (key, row) pairs, +inf padding)
    const int M = (int)min(N, (int64_t)kSortMax);
    int P = 1;
    while (P < M) P <<= 1;
    for (int i = tid; i < P; i += kBlock) {
        double s = INFINITY;
        if (i < M) {
            s = 0.0;
            for (int g = 0; g < G; ++g) s += (double)xd[(size_t)i * G + g];
        }
        key[i] = s;
        rid[i] = i;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P; i += kBlock) {
                const int p = i ^ j;
                if (p > i) {
                    const double ka = key[i], kc = key[p];
                    const int ia = rid[i], ic = rid[p];
                    const bool gt = ka > kc || (ka == kc && ia > ic);
                    if (gt == ((i & k) == 0)) {
                        key[i] = kc;
                        key[p] = ka;
                        rid[i] = ic;
                        rid[p] = ia;
                    }
                }
            }
            __syncthreads();
        }
    }
    // rank-bin means of every gene, summed in rank order
    for (int q = tid; q < 16 * G; q += kBlock) {
        const int g = q % G, j = q / G;
        const int lo = (int)(((int64_t)j * M) / 16);
        const int hi = max((int)(((int64_t)(j + 1) * M) / 16), lo + 1);
        double s = 0.0;
        for (int r = lo; r < hi; ++r) s += (double)xd[(size_t)rid[r] * G + g];
        f[(size_t)g * 18 + 2 + j] = (float)((s / (double)(hi - lo) - 25.0) / 10.0);
    }
}

// Nearest-rank quantiles of every gene, slots 2..17: q_j = sorted(x_g)[floor((j + 0.5) N / 16)],
// stored as (q_j - 25) / 10.  Exact order statistics by radix selection on the order-preserving
// 32-bit key of the floats, 4 bits per pass from the top, for a block of up to 32 genes at a time
// and all 16 ranks at once: the 16 order statistics of a gene are nondecreasing, so ranks that
// share the bits chosen so far form runs, and each value adds to the histogram of the run (if
// any) whose prefix it matches, found by a binary search over the 16 prefixes.
__device__ __forceinline__ uint32_t order_key(float v)
{
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_value(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

constexpr int kQGenes = 32;  // genes per block of the quantile search

__device__ void feature_quantiles(const float *__restrict__ xd, int64_t N, int G, float *__restrict__ f)
{
    __shared__ uint32_t hist[kQGenes][16][16];
    __shared__ uint32_t pref[kQGenes][16], npref[kQGenes][16];
    __shared__ int32_t rk[kQGenes][16], nrk[kQGenes][16];
    const int tid = threadIdx.x;
    for (int gb0 = 0; gb0 < G; gb0 += kQGenes) {
        const int ng = min(kQGenes, G - gb0);
        for (int i = tid; i < ng * 16; i += kBlock) {
            const int g = i >> 4, t = i & 15;
            pref[g][t] = 0u;
            rk[g][t] = (int32_t)floor(((double)t + 0.5) / 16.0 * (double)N);
        }
        __syncthreads();
        const int RP = kBlock / ng;  // row phases: lanes over the block's genes, coalesced along rows
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 28 - 4 * pass;
            const uint32_t hmask = pass == 0 ? 0u : (0xFFFFFFFFu << (shift + 4));
            for (int i = tid; i < ng * 256; i += kBlock) (&hist[0][0][0])[i] = 0u;
            __syncthreads();
            if (tid < RP * ng) {
                const int g = tid % ng, rp = tid / ng;
                for (int64_t n = rp; n < N; n += RP) {
                    const uint32_t key = order_key(xd[n * G + gb0 + g]);
                    const uint32_t mk = key & hmask;
                    int lo = 0;  // first rank whose prefix is >= mk
#pragma unroll
                    for (int step = 8; step > 0; step >>= 1)
                        if (pref[g][lo + step - 1] < mk) lo += step;
                    if (lo < 16 && pref[g][lo] == mk) atomicAdd(&hist[g][lo][(key >> shift) & 15u], 1u);
                }
            }
            __syncthreads();
            for (int i = tid; i < ng * 16; i += kBlock) {
                const int g = i >> 4, t = i & 15;
                int r0 = t;  // first rank of the run
                while (r0 > 0 && pref[g][r0 - 1] == pref[g][t]) --r0;
                uint32_t cum = 0;
                int dgt = 0;
                for (; dgt < 15; ++dgt) {
                    const uint32_t c = hist[g][r0][dgt];
                    if ((uint32_t)rk[g][t] < cum + c) break;
                    cum += c;
                }
                npref[g][t] = pref[g][t] | ((uint32_t)dgt << shift);
                nrk[g][t] = rk[g][t] - (int32_t)cum;
            }
            __syncthreads();
            for (int i = tid; i < ng * 16; i += kBlock) {
                const int g = i >> 4, t = i & 15;
                pref[g][t] = npref[g][t];
                rk[g][t] = nrk[g][t];
            }
            __syncthreads();
        }
        for (int i = tid; i < ng * 16; i += kBlock) {
            const int g = i >> 4, t = i & 15;
            f[(size_t)(gb0 + g) * 18 + 2 + t] = (float)(((double)key_value(pref[g][t]) - 25.0) / 10.0);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_features_q(const float *__restrict__ x, const int64_t *__restrict__ row_off,
                                                       int G, float *__restrict__ feat)
{
    const int b = blockIdx.x, tid = threadIdx.x;
    const int64_t r0 = row_off[b], N = row_off[b + 1] - r0;
    const float *xd = x + r0 * G;
    float *f = feat + (size_t)b * 18 * G;
    if (N <= 0) {
        for (int q = tid; q < 18 * G; q += kBlock) f[q] = NAN;
        return;
    }
    feature_moments(xd, N, G, f);
    feature_quantiles(xd, N, G, f);
}

// targets: one thread per dataset
__global__ void k_targets(const double *__restrict__ pi, const double *__restrict__ mu,
                          const double *__restrict__ tau, int B, int K, int G, float *__restrict__ tgt)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    int order[kMaxK];
    double key[kMaxK];
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) s += mu[((size_t)b * K + k) * G + g];
        key[k] = s / G;
        order[k] = k;
    }
    for (int i = 1; i < K; ++i) {  // insertion sort by (mean, index)
        const int o = order[i];
        int j = i - 1;
        while (j >= 0 && key[order[j]] > key[o]) {
            order[j + 1] = order[j];
            --j;
        }
        order[j + 1] = o;
    }
    const size_t KG = (size_t)K * G;
    float *t = tgt + (size_t)b * (2 * KG + K);
    for (int sl = 0; sl < K; ++sl) {
        const int k = order[sl];
        for (int g = 0; g < G; ++g) {
            t[(size_t)sl * G + g] = (float)((mu[((size_t)b * K + k) * G + g] - 25.0) / 10.0);
            t[KG + (size_t)sl * G + g] = (float)log(tau[((size_t)b * K + k) * G + g]);
        }
        t[2 * KG + sl] = (float)log(pi[(size_t)b * K + k]);
    }
}

// ---------------------------------------------------------------------------------------------
// C[M x N] = op(A)[M x K] op(B)[K x N] (+ bias[N]); optional GELU into Y (Z keeps the
// pre-activation).  op(A)[m][k] = TA ? A[k lda + m] : A[m lda + k];
// op(B)[k][n] = TB ? B[n ldb + k] : B[k ldb + n].  Operands are rounded to BF16 as
// they are staged in LDS; products accumulate in FP32 on MFMA 16x16x32.
// 256 threads: 4 waves, each a 32 x 32 sub-tile (2 x 2 MFMA tiles).
template <bool TA, bool TB>
__global__ __launch_bounds__(kBlock) void k_gemm(int M, int N, int K, const float *__restrict__ A, int lda,
                                                 const float *__restrict__ B, int ldb, const float *__restrict__ bias,
                                                 float *__restrict__ Z, float *__restrict__ Y, int ldc, int act)
{
    __shared__ __bf16 As[kTM][kTK + 8];  // [m][k]
    __shared__ __bf16 Bs[kTN][kTK + 8];  // [n][k]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += kTK) {
        for (int e = tid; e < kTM * kTK; e += kBlock) {
            int mm, kk;
            if (TA) {
                mm = e % kTM;
                kk = e / kTM;
            } else {
                kk = e % kTK;
                mm = e / kTK;
            }
            const int m = m0 + mm, k = k0 + kk;
            float v = 0.f;
            if (m < M && k < K) v = TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
            As[mm][kk] = to_bf16(v);
        }
        for (int e = tid; e < kTN * kTK; e += kBlock) {
            int nn, kk;
            if (TB) {
                kk = e % kTK;
                nn = e / kTK;
            } else {
                nn = e % kTN;
                kk = e / kTN;
            }
            const int n = n0 + nn, k = k0 + kk;
            float v = 0.f;
            if (n < N && k < K) v = TB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
            Bs[nn][kk] = to_bf16(v);
        }
        __syncthreads();
        const int r = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            bf16x8 a;
#pragma unroll
            for (int t = 0; t < 8; ++t) a[t] = As[wm + 16 * i + r][kq + t];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                bf16x8 bb;
#pragma unroll
                for (int t = 0; t < 8; ++t) bb[t] = Bs[wn + 16 * j + r][kq + t];
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // lane holds rows 4 (lane / 16) + e, column lane % 16 of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + e;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m < M && n < N) {
                    float z = acc[i][j][e] + (bias ? bias[n] : 0.f);
                    Z[(size_t)m * ldc + n] = z;
                    if (Y) Y[(size_t)m * ldc + n] = act ? gelu(z) : z;
                }
            }
}

// dZ = dY * gelu'(Z), elementwise
__global__ void k_gelu_back(int n, const float *__restrict__ Z, const float *__restrict__ dY, float *__restrict__ dZ)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dZ[i] = dY[i] * gelu_grad(Z[i]);
}

// column sums of a M x N matrix (fixed order per column)
__global__ void k_colsum(int M, int N, const float *__restrict__ D, float *__restrict__ out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double s = 0.0;
    for (int m = 0; m < M; ++m) s += (double)D[(size_t)m * N + n];
    out[n] = (float)s;
}

// mean squared error and its gradient dY = 2 (Y - T) / (M N); per-block FP64 partial losses
__global__ void k_mse(int n, float scale, const float *__restrict__ Y, const float *__restrict__ T,
                      float *__restrict__ dY, double *__restrict__ part)
{
    __shared__ double red[kBlock];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double l = 0.0;
    if (i < n) {
        const float d = Y[i] - T[i];
        dY[i] = 2.0f * d * scale;
        l = (double)d * (double)d;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// AdamW on FP32 master parameters
__global__ void k_adamw(int64_t n, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                        float *__restrict__ v, float lr, float b1, float b2, float eps, float wd, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    w[i] -= lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
}

// MLP output rows -> variational state of each dataset of a batch (its own K):
//   pi = softmax(log pi), alpha = alpha0 + N pi, beta = beta0 + N pi_k,
//   m = 25 + 10 mhat, a = a0 + N pi_k / 2, b = a / exp(ln tau).
__global__ void k_warm_state(Shape s, Bufs bf, Prior p, const float *__restrict__ out, int ld)
{
    const int bi = blockIdx.x, tid = threadIdx.x, G = s.G;
    const Ds d = bf.ds[bi];
    const int K = d.K;
    const float *o = out + (size_t)bi * ld;
    const size_t kb = (size_t)bi * s.Kmax, kg = kb * G;
    __shared__ double pk[kMaxK];
    if (tid == 0) {
        double mx = -INFINITY;
        for (int k = 0; k < K; ++k) mx = fmax(mx, (double)o[2 * K * G + k]);
        double se = 0.0;
        for (int k = 0; k < K; ++k) se += exp((double)o[2 * K * G + k] - mx);
        for (int k = 0; k < K; ++k) pk[k] = exp((double)o[2 * K * G + k] - mx) / se;
    }
    __syncthreads();
    if (tid < K) bf.alpha[kb + tid] = p.alpha0 + d.N * pk[tid];
    for (int q = tid; q < K * G; q += kBlock) {
        const int k = q / G;
        const double nk = d.N * pk[k];
        const double a = p.a0 + 0.5 * nk;
        const double lt = fmin(fmax((double)o[K * G + q], -30.0), 30.0);
        bf.m[kg + q] = 25.0 + 10.0 * (double)o[q];
        bf.beta[kg + q] = p.beta0 + nk;
        bf.a[kg + q] = a;
        bf.b[kg + q] = a / exp(lt);
    }
}

// Each dataset's state as a row of the warm-start layout that k_warm_state reads back: (m - 25) / 10
// [K G] | ln(a / b) [K G] | ln max(alpha - alpha0, 1/2) [K] (the counts N_k, floored at half a row
// so that an emptied subpopulation does not dominate a regression on these rows; their softmax is
// E[pi]), then, with centre, (m0_g - 25) / 10 [G].  One workgroup per dataset.
__global__ void k_state_rows(Shape s, Bufs bf, Prior p, float *__restrict__ rows, int ld, int centre)
{
    const int bi = blockIdx.x, tid = threadIdx.x, G = s.G;
    const int K = bf.ds[bi].K;
    float *o = rows + (size_t)bi * ld;
    const size_t kb = (size_t)bi * s.Kmax, kg = kb * G;
    for (int q = tid; q < K * G; q += kBlock) {
        o[q] = (float)((bf.m[kg + q] - 25.0) / 10.0);
        o[K * G + q] = (float)log(bf.a[kg + q] / bf.b[kg + q]);
    }
    if (tid < K) o[2 * K * G + tid] = (float)log(fmax(bf.alpha[kb + tid] - p.alpha0, 0.5));
    if (centre)
        for (int g = tid; g < G; g += kBlock) o[K * (2 * G + 1) + g] = (float)((bf.m0[(size_t)bi * G + g] - 25.0) / 10.0);
}

// y[i][j] += alpha x[i][j] for i < n, j < m (row strides ldx, ldy)
__global__ void k_rows_axpy(int n, int m, float alpha, const float *__restrict__ x, int ldx, float *__restrict__ y,
                            int ldy)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * m) return;
    const int i = (int)(t / m), j = (int)(t - (int64_t)i * m);
    y[(size_t)i * ldy + j] = fmaf(alpha, x[(size_t)i * ldx + j], y[(size_t)i * ldy + j]);
}

// ---------------------------------------------------------------------------------------------
hipError_t launch_state_rows(const Shape &s, const Bufs &b, const Prior &p, float *rows, int ld, int centre,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_state_rows, dim3(s.B), dim3(kBlock), 0, st, s, b, p, rows, ld, centre);
    return hipGetLastError();
}

hipError_t launch_rows_axpy(int n, int m, float alpha, const float *x, int ldx, float *y, int ldy, hipStream_t st)
{
    const int64_t tot = (int64_t)n * m;
    hipLaunchKernelGGL(k_rows_axpy, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, m, alpha,
                       x, ldx, y, ldy);
    return hipGetLastError();
}

hipError_t launch_features(const float *x, const int64_t *row_off, int B, int G, float *feat, hipStream_t st)
{
    hipLaunchKernelGGL(k_features, dim3(B), dim3(kBlock), 0, st, x, row_off, G, feat);
    return hipGetLastError();
}

hipError_t launch_features_quantiles(const float *x, const int64_t *row_off, int B, int G, float *feat, hipStream_t st)
{
    hipLaunchKernelGGL(k_features_q, dim3(B), dim3(kBlock), 0, st, x, row_off, G, feat);
    return hipGetLastError();
}

hipError_t launch_targets(const double *pi, const double *mu, const double *tau, int B, int K, int G, float *tgt,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_targets, dim3((B + 63) / 64), dim3(64), 0, st, pi, mu, tau, B, K, G, tgt);
    return hipGetLastError();
}

hipError_t launch_gemm(bool ta, bool tb, int M, int N, int K, const float *A, int lda, const float *B, int ldb,
                       const float *bias, float *Z, float *Y, int ldc, int act, hipStream_t st)
{
    const dim3 grid((N + kTN - 1) / kTN, (M + kTM - 1) / kTM);
    if (!ta && !tb)
        hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(kBlock), 0, st, M, N, K, A, lda, B, ldb, bias, Z, Y, ldc, act);
    else if (!ta && tb)
        hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(kBlock), 0, st, M, N, K, A, lda, B, ldb, bias, Z, Y, ldc, act);
    else if (ta && !tb)
        hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(kBlock), 0, st, M, N, K, A, lda, B, ldb, bias, Z, Y, ldc, act);
    else
        hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(kBlock), 0, st, M, N, K, A, lda, B, ldb, bias, Z, Y, ldc, act);
    return hipGetLastError();
}

hipError_t launch_gelu_back(int n, const float *Z, const float *dY, float *dZ, hipStream_t st)
{
    hipLaunchKernelGGL(k_gelu_back, dim3((n + 255) / 256), dim3(256), 0, st, n, Z, dY, dZ);
    return hipGetLastError();
}

hipError_t launch_colsum(int M, int N, const float *D, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, st, M, N, D, out);
    return hipGetLastError();
}

hipError_t launch_mse(int n, float scale, const float *Y, const float *T, float *dY, double *part, hipStream_t st)
{
    hipLaunchKernelGGL(k_mse, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, n, scale, Y, T, dY, part);
    return hipGetLastError();
}

hipError_t launch_adamw(int64_t n, float *w, const float *g, float *m, float *v, float lr, float b1, float b2,
                        float eps, float wd, float c1, float c2, hipStream_t st)
{
    hipLaunchKernelGGL(k_adamw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, w, g, m, v, lr, b1, b2, eps,
                       wd, c1, c2);
    return hipGetLastError();
}

hipError_t launch_warm_state(const Shape &s, const Bufs &b, const Prior &p, const float *out, int ld, hipStream_t st)
{
    hipLaunchKernelGGL(k_warm_state, dim3(s.B), dim3(kBlock), 0, st, s, b, p, out, ld);
    return hipGetLastError();
}

}  // namespace cavi
