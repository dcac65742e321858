// Host side of the learned warm start: features, training targets, and the
// MLP (parameters, forward, loss gradient, AdamW) behind include/cavi.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "../../include/cavi.h"
#include "cavi_impl.h"

using namespace cavi;

namespace {

cavi_status wfail(cavi_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_last_error(buf);
    return st;
}

#define WCHK(expr)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return wfail(CAVI_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

}  // namespace

struct cavi_mlp {
    int L = 0;                   // linear layers
    std::vector<int> dims;       // L + 1
    std::vector<int64_t> offW, offb;
    int64_t nparams = 0;
    int max_batch = 0;
    int step = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    std::vector<float *> Z, Y;   // per layer, max_batch x dims[l]
    std::vector<float *> dZ;     // per layer, max_batch x dims[l]: gradient of the loss w.r.t. Z_l
    double *part = nullptr;
    int npart = 0;
};

extern "C" {

cavi_status cavi_features(const float *x_dev, const int64_t *row_off_dev, int32_t B, int32_t G, float *feat_dev,
                          void *hip_stream)
{
    if (!x_dev || !row_off_dev || !feat_dev) return wfail(CAVI_E_INVAL, "NULL argument");
    if (B < 1 || G < 1 || G > kMaxG) return wfail(CAVI_E_INVAL, "B=%d, G=%d out of range", B, G);
    WCHK(launch_features(x_dev, row_off_dev, B, G, feat_dev, (hipStream_t)hip_stream));
    return CAVI_OK;
}

cavi_status cavi_features_quantiles(const float *x_dev, const int64_t *row_off_dev, int32_t B, int32_t G,
                                    float *feat_dev, void *hip_stream)
{
    if (!x_dev || !row_off_dev || !feat_dev) return wfail(CAVI_E_INVAL, "NULL argument");
    if (B < 1 || G < 1 || G > kMaxG) return wfail(CAVI_E_INVAL, "B=%d, G=%d out of range", B, G);
    WCHK(launch_features_quantiles(x_dev, row_off_dev, B, G, feat_dev, (hipStream_t)hip_stream));
    return CAVI_OK;
}

cavi_status cavi_rows_axpy(int32_t n, int32_t m, float alpha, const float *x_dev, int32_t ldx, float *y_dev,
                           int32_t ldy, void *hip_stream)
{
    if (!x_dev || !y_dev) return wfail(CAVI_E_INVAL, "NULL argument");
    if (n < 1 || m < 1 || ldx < m || ldy < m) return wfail(CAVI_E_INVAL, "n=%d, m=%d, ldx=%d, ldy=%d", n, m, ldx, ldy);
    WCHK(launch_rows_axpy(n, m, alpha, x_dev, ldx, y_dev, ldy, (hipStream_t)hip_stream));
    return CAVI_OK;
}

cavi_status cavi_warm_targets(const double *pi_dev, const double *mu_dev, const double *tau_dev, int32_t B,
                              int32_t K, int32_t G, float *target_dev, void *hip_stream)
{
    if (!pi_dev || !mu_dev || !tau_dev || !target_dev) return wfail(CAVI_E_INVAL, "NULL argument");
    if (B < 1 || K < 1 || K > kMaxK || G < 1) return wfail(CAVI_E_INVAL, "B=%d, K=%d, G=%d out of range", B, K, G);
    WCHK(launch_targets(pi_dev, mu_dev, tau_dev, B, K, G, target_dev, (hipStream_t)hip_stream));
    return CAVI_OK;
}

cavi_status cavi_mlp_destroy(cavi_mlp *net)
{
    if (!net) return CAVI_OK;
    if (net->stream) (void)hipStreamSynchronize(net->stream);
    for (float *p : {net->params, net->grads, net->m, net->v})
        if (p) (void)hipFree(p);
    for (const std::vector<float *> *a : {&net->Z, &net->Y, &net->dZ})
        for (float *p : *a)
            if (p) (void)hipFree(p);
    if (net->part) (void)hipFree(net->part);
    if (net->own_stream && net->stream) (void)hipStreamDestroy(net->stream);
    delete net;
    return CAVI_OK;
}

cavi_status cavi_mlp_create(cavi_mlp **out, int32_t in_dim, int32_t hidden, int32_t n_hidden, int32_t out_dim,
                            int32_t max_batch, uint64_t seed, void *hip_stream)
{
    if (!out) return wfail(CAVI_E_INVAL, "out is NULL");
    *out = nullptr;
    if (in_dim < 1 || hidden < 1 || n_hidden < 0 || out_dim < 1 || max_batch < 1)
        return wfail(CAVI_E_INVAL, "bad MLP dimensions");
    cavi_mlp *n = new cavi_mlp;
    n->L = n_hidden + 1;
    n->dims.push_back(in_dim);
    for (int i = 0; i < n_hidden; ++i) n->dims.push_back(hidden);
    n->dims.push_back(out_dim);
    n->max_batch = max_batch;
    for (int l = 0; l < n->L; ++l) {
        n->offW.push_back(n->nparams);
        n->nparams += (int64_t)n->dims[l + 1] * n->dims[l];
        n->offb.push_back(n->nparams);
        n->nparams += n->dims[l + 1];
    }
    // parameters: W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from SplitMix64(seed), b = 0
    std::vector<float> host(n->nparams, 0.f);
    uint64_t s = seed;
    for (int l = 0; l < n->L; ++l) {
        const double lim = 1.0 / sqrt((double)n->dims[l]);
        const int64_t cnt = (int64_t)n->dims[l + 1] * n->dims[l];
        for (int64_t i = 0; i < cnt; ++i) {
            const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
            host[n->offW[l] + i] = (float)((2.0 * u - 1.0) * lim);
        }
    }
    hipError_t e = hipSuccess;
    // NULL: the default stream, which orders the network's work with the caller's default-stream
    // work and with the CAVI handles' own streams (they are blocking streams)
    n->stream = (hipStream_t)hip_stream;
    const size_t pb = sizeof(float) * n->nparams;
    if (e == hipSuccess) e = hipMalloc(&n->params, pb);
    if (e == hipSuccess) e = hipMalloc(&n->grads, pb);
    if (e == hipSuccess) e = hipMalloc(&n->m, pb);
    if (e == hipSuccess) e = hipMalloc(&n->v, pb);
    for (int l = 0; l <= n->L && e == hipSuccess; ++l) {
        float *z = nullptr, *y = nullptr, *dz = nullptr;
        e = hipMalloc(&z, sizeof(float) * (size_t)max_batch * n->dims[l]);
        if (e == hipSuccess) e = hipMalloc(&y, sizeof(float) * (size_t)max_batch * n->dims[l]);
        if (e == hipSuccess) e = hipMalloc(&dz, sizeof(float) * (size_t)max_batch * n->dims[l]);
        n->Z.push_back(z);
        n->Y.push_back(y);
        n->dZ.push_back(dz);
    }
    n->npart = (int)(((int64_t)max_batch * out_dim + kBlock - 1) / kBlock);
    if (e == hipSuccess) e = hipMalloc(&n->part, sizeof(double) * n->npart);
    if (e == hipSuccess) e = hipMemcpyAsync(n->params, host.data(), pb, hipMemcpyHostToDevice, n->stream);
    if (e == hipSuccess) e = hipMemsetAsync(n->m, 0, pb, n->stream);
    if (e == hipSuccess) e = hipMemsetAsync(n->v, 0, pb, n->stream);
    if (e == hipSuccess) e = hipMemsetAsync(n->grads, 0, pb, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        cavi_mlp_destroy(n);
        return wfail(CAVI_E_NOMEM, "MLP allocation: %s", hipGetErrorString(e));
    }
    *out = n;
    return CAVI_OK;
}

cavi_status cavi_mlp_n_params(cavi_mlp *net, int64_t *n)
{
    if (!net || !n) return wfail(CAVI_E_INVAL, "NULL argument");
    *n = net->nparams;
    return CAVI_OK;
}

cavi_status cavi_mlp_get_params(cavi_mlp *net, float *host)
{
    if (!net || !host) return wfail(CAVI_E_INVAL, "NULL argument");
    WCHK(hipMemcpyAsync(host, net->params, sizeof(float) * net->nparams, hipMemcpyDeviceToHost, net->stream));
    WCHK(hipStreamSynchronize(net->stream));
    return CAVI_OK;
}

cavi_status cavi_mlp_set_params(cavi_mlp *net, const float *host)
{
    if (!net || !host) return wfail(CAVI_E_INVAL, "NULL argument");
    WCHK(hipMemcpyAsync(net->params, host, sizeof(float) * net->nparams, hipMemcpyHostToDevice, net->stream));
    WCHK(hipStreamSynchronize(net->stream));
    return CAVI_OK;
}

cavi_status cavi_mlp_get_grads(cavi_mlp *net, float *host)
{
    if (!net || !host) return wfail(CAVI_E_INVAL, "NULL argument");
    WCHK(hipMemcpyAsync(host, net->grads, sizeof(float) * net->nparams, hipMemcpyDeviceToHost, net->stream));
    WCHK(hipStreamSynchronize(net->stream));
    return CAVI_OK;
}

static cavi_status forward(cavi_mlp *n, const float *feat, int B, float *out_last)
{
    const float *in = feat;
    for (int l = 0; l < n->L; ++l) {
        const int K = n->dims[l], N = n->dims[l + 1];
        const bool last = l == n->L - 1;
        float *y = last ? (out_last ? out_last : n->Y[l + 1]) : n->Y[l + 1];
        WCHK(launch_gemm(false, true, B, N, K, in, K, n->params + n->offW[l], K, n->params + n->offb[l],
                         n->Z[l + 1], y, N, last ? 0 : 1, n->stream));
        in = y;
    }
    return CAVI_OK;
}

cavi_status cavi_mlp_forward(cavi_mlp *net, const float *feat_dev, int32_t B, float *out_dev)
{
    if (!net || !feat_dev || !out_dev) return wfail(CAVI_E_INVAL, "NULL argument");
    if (B < 1 || B > net->max_batch) return wfail(CAVI_E_INVAL, "B=%d outside [1, %d]", B, net->max_batch);
    return forward(net, feat_dev, B, out_dev);
}

cavi_status cavi_mlp_loss_grad(cavi_mlp *net, const float *feat_dev, const float *target_dev, int32_t B,
                               float *loss_host)
{
    if (!net || !feat_dev || !target_dev) return wfail(CAVI_E_INVAL, "NULL argument");
    if (B < 1 || B > net->max_batch) return wfail(CAVI_E_INVAL, "B=%d outside [1, %d]", B, net->max_batch);
    cavi_mlp *n = net;
    cavi_status st = forward(n, feat_dev, B, nullptr);
    if (st != CAVI_OK) return st;
    const int L = n->L, O = n->dims[L];
    const int cnt = B * O;
    WCHK(launch_mse(cnt, 1.0f / (float)cnt, n->Y[L], target_dev, n->dZ[L], n->part, n->stream));
    for (int l = L - 1; l >= 0; --l) {
        const int K = n->dims[l], N = n->dims[l + 1];
        const float *in = l == 0 ? feat_dev : n->Y[l];
        const float *dZ = n->dZ[l + 1];
        // dW = dZ^T X  [N x K];  db = column sums of dZ
        WCHK(launch_gemm(true, false, N, K, B, dZ, N, in, K, nullptr, n->grads + n->offW[l], nullptr, K, 0,
                         n->stream));
        WCHK(launch_colsum(B, N, dZ, n->grads + n->offb[l], n->stream));
        if (l > 0) {
            // dY = dZ W  [B x K], then through the GELU of layer l (in place)
            WCHK(launch_gemm(false, false, B, K, N, dZ, N, n->params + n->offW[l], K, nullptr, n->dZ[l], nullptr,
                             K, 0, n->stream));
            WCHK(launch_gelu_back(B * K, n->Z[l], n->dZ[l], n->dZ[l], n->stream));
        }
    }
    if (loss_host) {
        const int np = (cnt + kBlock - 1) / kBlock;
        std::vector<double> part(np);
        WCHK(hipMemcpyAsync(part.data(), n->part, sizeof(double) * np, hipMemcpyDeviceToHost, n->stream));
        WCHK(hipStreamSynchronize(n->stream));
        double s = 0.0;
        for (double p : part) s += p;
        *loss_host = (float)(s / cnt);
    }
    return CAVI_OK;
}

cavi_status cavi_mlp_get_layer(cavi_mlp *net, int32_t layer, int32_t what, int32_t B, float *host)
{
    if (!net || !host) return wfail(CAVI_E_INVAL, "NULL argument");
    if (layer < 1 || layer > net->L) return wfail(CAVI_E_INVAL, "layer=%d outside [1, %d]", layer, net->L);
    if (what < 0 || what > 2) return wfail(CAVI_E_INVAL, "what=%d outside [0, 2]", what);
    if (B < 1 || B > net->max_batch) return wfail(CAVI_E_INVAL, "B=%d outside [1, %d]", B, net->max_batch);
    const float *src = what == 0 ? net->Z[layer] : what == 1 ? net->Y[layer] : net->dZ[layer];
    WCHK(hipMemcpyAsync(host, src, sizeof(float) * (size_t)B * net->dims[layer], hipMemcpyDeviceToHost,
                        net->stream));
    WCHK(hipStreamSynchronize(net->stream));
    return CAVI_OK;
}

cavi_status cavi_mlp_adamw(cavi_mlp *net, float lr, float beta1, float beta2, float eps, float weight_decay)
{
    if (!net) return wfail(CAVI_E_INVAL, "net is NULL");
    net->step += 1;
    const float c1 = 1.0f - powf(beta1, (float)net->step), c2 = 1.0f - powf(beta2, (float)net->step);
    WCHK(launch_adamw(net->nparams, net->params, net->grads, net->m, net->v, lr, beta1, beta2, eps, weight_decay, c1,
                      c2, net->stream));
    return CAVI_OK;
}

}  // extern "C"
