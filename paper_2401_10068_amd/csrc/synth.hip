// On-device twin of the seeded input generator defined in synth.py
// (Philox4x32-10 bits, Box--Muller normals, Marsaglia--Tsang Gamma draws,
// Dirichlet proportions, Gaussian-mixture rows).  An input generator only:
// nothing of the inference arithmetic is here.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace {

constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
constexpr uint32_t kStreamParams = 0, kStreamLabel = 1, kStreamNormal = 2;
constexpr double kTwoM53 = 1.1102230246251565404236316680908203125e-16;  // 2^-53
constexpr double kPi = 3.141592653589793115997963468544185161590576171875;

struct W4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ W4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kM0 * c0;
        const uint64_t p1 = (uint64_t)kM1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += kW0;
        k1 += kW1;
    }
    return W4{c0, c1, c2, c3};
}

__device__ __forceinline__ double u53(uint32_t lo, uint32_t hi)
{
    const uint64_t m = ((((uint64_t)hi) << 32) | lo) >> 11;
    return ((double)m + 0.5) * kTwoM53;
}

struct ParamStream {
    uint32_t k0, k1;
    uint64_t index;

    __device__ W4 block()
    {
        const uint64_t i = index++;
        return philox((uint32_t)i, (uint32_t)(i >> 32), 0, kStreamParams, k0, k1);
    }
    __device__ double uniform()
    {
        const W4 w = block();
        return u53(w.w0, w.w1);
    }
    __device__ double normal()
    {
#pragma clang fp contract(off)
        const W4 w = block();
        const double u1 = u53(w.w0, w.w1), u2 = u53(w.w2, w.w3);
        return sqrt(-2.0 * log(u1)) * cos(2.0 * kPi * u2);
    }
    __device__ double gamma_ge1(double shape, double rate)
    {
#pragma clang fp contract(off)
        const double d = shape - 1.0 / 3.0;
        const double c = 1.0 / sqrt(9.0 * d);
        for (;;) {
            const double u = uniform();
            const double n = normal();
            const double t = 1.0 + c * n;
            const double v = t * t * t;
            if (v > 0.0 && log(u) < 0.5 * n * n + d - d * v + d * log(v)) return d * v / rate;
        }
    }
    __device__ double gamma(double shape, double rate)
    {
#pragma clang fp contract(off)
        if (shape < 1.0) {
            const double g = gamma_ge1(shape + 1.0, 1.0);
            const double u = uniform();
            return g * pow(u, 1.0 / shape) / rate;
        }
        return gamma_ge1(shape, rate);
    }
};

// One thread per dataset: proportions, means and precisions in the
// generator's draw order.
__global__ void k_params(uint32_t seed, int B, int ds_offset, const int *__restrict__ Kb, int Kmax, int G,
                         double dir_alpha, double mu_lo, double mu_hi, double tau_shape, double tau_rate,
                         int overlap_pairs, double overlap_sd, double *__restrict__ pi,
                         double *__restrict__ mu, double *__restrict__ tau)
{
#pragma clang fp contract(off)
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int K = Kb[b];
    ParamStream st{seed, (uint32_t)(ds_offset + b), 0};
    double *pib = pi + (size_t)b * Kmax;
    double *mub = mu + (size_t)b * Kmax * G;
    double *taub = tau + (size_t)b * Kmax * G;
    double s = 0.0;
    for (int k = 0; k < K; ++k) {
        pib[k] = st.gamma(dir_alpha, 1.0);
        s += pib[k];
    }
    for (int k = 0; k < K; ++k) pib[k] = pib[k] / s;
    for (int k = K; k < Kmax; ++k) pib[k] = 0.0;
    for (int k = 0; k < K; ++k)
        for (int g = 0; g < G; ++g) {
            mub[k * G + g] = mu_lo + (mu_hi - mu_lo) * st.uniform();
            taub[k * G + g] = st.gamma(tau_shape, tau_rate);
        }
    const int pairs = min(overlap_pairs, K / 2);
    for (int j = 0; j < pairs; ++j)
        for (int g = 0; g < G; ++g) {
            const int a = (2 * j) * G + g, c = (2 * j + 1) * G + g;
            taub[c] = taub[a];
            mub[c] = mub[a] + overlap_sd / sqrt(taub[a]);
        }
}

// One thread per (row, gene pair) over the concatenated rows of B datasets.
__global__ void k_rows(uint32_t seed, int B, int ds_offset, const int64_t *__restrict__ row_off,
                       const int *__restrict__ Kb, int Kmax, int G, const double *__restrict__ pi,
                       const double *__restrict__ mu, const double *__restrict__ tau, float *__restrict__ x,
                       int *__restrict__ z, int64_t total_rows)
{
#pragma clang fp contract(off)
    const int npair = (G + 1) / 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total_rows * npair) return;
    const int64_t grow = t / npair;
    const int j = (int)(t - grow * npair);
    int lo = 0, hi = B;  // row_off[lo] <= grow < row_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (row_off[mid] <= grow) lo = mid;
        else hi = mid;
    }
    const int b = lo;
    const int64_t row = grow - row_off[b];
    const uint32_t k0 = seed, k1 = (uint32_t)(ds_offset + b);
    const int K = Kb[b];
    const double *pib = pi + (size_t)b * Kmax;
    const W4 wl = philox((uint32_t)row, (uint32_t)(row >> 32), 0, kStreamLabel, k0, k1);
    const double u = u53(wl.w0, wl.w1);
    double cum = 0.0;
    int zz = 0;
    for (int k = 0; k < K; ++k) {
        cum += pib[k];
        if (cum <= u) zz = k + 1;
    }
    if (zz > K - 1) zz = K - 1;
    if (z && j == 0) z[grow] = zz;
    const W4 w = philox((uint32_t)row, (uint32_t)(row >> 32), (uint32_t)j, kStreamNormal, k0, k1);
    const double u1 = u53(w.w0, w.w1), u2 = u53(w.w2, w.w3);
    const double rad = sqrt(-2.0 * log(u1));
    const double th = 2.0 * kPi * u2;
    const double *mub = mu + ((size_t)b * Kmax + zz) * G;
    const double *taub = tau + ((size_t)b * Kmax + zz) * G;
    const int g0 = 2 * j;
    float *xr = x + grow * G;
    {
        const double sd = 1.0 / sqrt(taub[g0]);
        xr[g0] = (float)(mub[g0] + (rad * cos(th)) * sd);
    }
    if (g0 + 1 < G) {
        const double sd = 1.0 / sqrt(taub[g0 + 1]);
        xr[g0 + 1] = (float)(mub[g0 + 1] + (rad * sin(th)) * sd);
    }
}

}  // namespace

extern "C" {

// Parameters of datasets ds_offset .. ds_offset+B-1 (device arrays; pi is
// B x Kmax, mu and tau are B x Kmax x G).  Returns a hipError_t code.
int synth_params(uint32_t seed, int32_t B, int32_t ds_offset, const int32_t *K_dev, int32_t Kmax, int32_t G,
                 double dir_alpha, double mu_lo, double mu_hi, double tau_shape, double tau_rate,
                 int32_t overlap_pairs, double overlap_sd, double *pi_dev, double *mu_dev, double *tau_dev,
                 void *stream)
{
    if (B <= 0) return 0;
    hipLaunchKernelGGL(k_params, dim3((B + 63) / 64), dim3(64), 0, (hipStream_t)stream, seed, B, ds_offset, K_dev,
                       Kmax, G, dir_alpha, mu_lo, mu_hi, tau_shape, tau_rate, overlap_pairs, overlap_sd, pi_dev,
                       mu_dev, tau_dev);
    return (int)hipGetLastError();
}

// Rows of the same datasets, concatenated (row_off has B+1 entries, first 0).
// x is total_rows x G FP32; z (int32 per row) may be NULL.
int synth_rows(uint32_t seed, int32_t B, int32_t ds_offset, const int64_t *row_off_dev, const int32_t *K_dev,
               int32_t Kmax, int32_t G, const double *pi_dev, const double *mu_dev, const double *tau_dev,
               float *x_dev, int32_t *z_dev, int64_t total_rows, void *stream)
{
    const int64_t work = total_rows * ((G + 1) / 2);
    if (work <= 0) return 0;
    const int64_t blocks = (work + 255) / 256;
    hipLaunchKernelGGL(k_rows, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, seed, B, ds_offset,
                       row_off_dev, K_dev, Kmax, G, pi_dev, mu_dev, tau_dev, x_dev, z_dev, total_rows);
    return (int)hipGetLastError();
}

}  // extern "C"
