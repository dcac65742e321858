// Host runtime behind include/cavi.h: argument checks, workspace, the
// k-means++ initialisation driver, hipGraph-captured sweeps, and the
// convergence loop.  All device work is in cavi_kernels.hip.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/cavi.h"
#include "cavi_impl.h"

using namespace cavi;

namespace {

thread_local std::string g_err;

cavi_status fail(cavi_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                                \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(CAVI_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

constexpr int kGraphSweeps = 16;  // sweeps per captured graph

// SplitMix64 (Steele, Lea and Flood 2014) and floor(u53 * n / 2^53).
uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t scaled_draw(uint64_t &s, uint64_t n)
{
    const uint64_t u = splitmix64(s) >> 11;
    return (uint64_t)(((unsigned __int128)u * (unsigned __int128)n) >> 53);
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

}  // namespace

struct cavi_ctx {
    Shape s{};
    Bufs b{};
    Prior p{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *ws = nullptr;
    bool own_ws = false;
    bool have_state = false;
    hipGraphExec_t graph = nullptr;
    Ctl *hctl = nullptr;  // pinned host mirror of the control block
};

extern "C" {

const char *cavi_last_error(void) { return g_err.c_str(); }

const char *cavi_version(void) { return "cavi-gfx950 0.1.0"; }

cavi_status cavi_prior_default(cavi_prior *prior)
{
    if (!prior) return fail(CAVI_E_INVAL, "prior is NULL");
    prior->alpha0 = 1.0;
    prior->beta0 = 1e-3;
    prior->a0 = 0.5;
    prior->b0 = 0.5;
    prior->m0 = nullptr;
    return CAVI_OK;
}

static cavi_status make_shape(int64_t N, int32_t G, int32_t K, Shape &s)
{
    if (K < 1 || K > kMaxK) return fail(CAVI_E_INVAL, "K=%d outside [1, %d]", K, kMaxK);
    if (G < 1 || G > kMaxG) return fail(CAVI_E_INVAL, "G=%d outside [1, %d]", G, kMaxG);
    if ((int64_t)K * G > kMaxKG) return fail(CAVI_E_INVAL, "K*G=%lld exceeds %d", (long long)K * G, kMaxKG);
    if (N < K) return fail(CAVI_E_INVAL, "N=%lld < K=%d", (long long)N, K);
    if (N >= ((int64_t)1 << 31)) return fail(CAVI_E_INVAL, "N=%lld too large", (long long)N);
    s.N = N;
    s.G = G;
    s.K = K;
    s.nchunk = (int32_t)((N + kChunkRows - 1) / kChunkRows);
    s.S = K + 2 * K * G + 1;
    s.kt = choose_kt(K);
    s.tile_rows = choose_tile_rows(G, s.kt);
    s.nblk = (int32_t)((N + kBlock - 1) / kBlock);
    return CAVI_OK;
}

cavi_status cavi_workspace_bytes(int64_t N, int32_t G, int32_t K, size_t *bytes)
{
    if (!bytes) return fail(CAVI_E_INVAL, "bytes is NULL");
    Shape s;
    cavi_status st = make_shape(N, G, K, s);
    if (st != CAVI_OK) return st;
    *bytes = workspace_bytes(s);
    return CAVI_OK;
}

cavi_status cavi_destroy(cavi_ctx *ctx)
{
    if (!ctx) return CAVI_OK;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
    if (ctx->own_ws && ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->hctl) (void)hipHostFree(ctx->hctl);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return CAVI_OK;
}

cavi_status cavi_create(cavi_ctx **out, const float *x_dev, int64_t N, int32_t G, int32_t K,
                        const cavi_prior *prior, void *hip_stream, void *workspace_dev, size_t ws_bytes)
{
    if (!out) return fail(CAVI_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!x_dev) return fail(CAVI_E_INVAL, "x_dev is NULL");
    if (((uintptr_t)x_dev) & 15) return fail(CAVI_E_INVAL, "x_dev is not 16-byte aligned");
    Shape s;
    cavi_status st = make_shape(N, G, K, s);
    if (st != CAVI_OK) return st;
    cavi_prior pr;
    cavi_prior_default(&pr);
    if (prior) pr = *prior;
    if (!finite_pos(pr.alpha0) || !finite_pos(pr.beta0) || !finite_pos(pr.a0) || !finite_pos(pr.b0))
        return fail(CAVI_E_INVAL, "prior hyperparameters must be finite and > 0");
    if (pr.m0)
        for (int g = 0; g < G; ++g)
            if (!isfinite(pr.m0[g])) return fail(CAVI_E_INVAL, "prior m0[%d] is not finite", g);
    const size_t need = workspace_bytes(s);
    if (workspace_dev) {
        if (ws_bytes < need) return fail(CAVI_E_NOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
        if (((uintptr_t)workspace_dev) & 255) return fail(CAVI_E_INVAL, "workspace is not 256-byte aligned");
    }
    hipError_t e = prepare_kernels();
    if (e != hipSuccess) return fail(CAVI_E_HIP, "device query: %s", hipGetErrorString(e));
    s.tile_rows = choose_tile_rows(G, s.kt);
    if (s.tile_rows < 16) return fail(CAVI_E_INVAL, "G=%d needs more LDS per block than the device has", G);
    cavi_ctx *c = new cavi_ctx;
    c->s = s;
    c->p = Prior{pr.alpha0, pr.beta0, pr.a0, pr.b0};
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreate(&c->stream);
        if (e != hipSuccess) {
            delete c;
            return fail(CAVI_E_HIP, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        c->own_stream = true;
    }
    if (workspace_dev) {
        c->ws = workspace_dev;
    } else {
        e = hipMalloc(&c->ws, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            cavi_destroy(c);
            return fail(CAVI_E_NOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
        }
        c->own_ws = true;
    }
    e = hipHostMalloc((void **)&c->hctl, sizeof(Ctl), hipHostMallocDefault);
    if (e != hipSuccess) {
        cavi_destroy(c);
        return fail(CAVI_E_HIP, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    carve(s, c->ws, c->b);
    c->b.x = x_dev;
    cavi_status rs = CAVI_OK;
    if (pr.m0) {
        e = hipMemcpyAsync(c->b.m0, pr.m0, sizeof(double) * G, hipMemcpyHostToDevice, c->stream);
    } else {
        e = launch_prior_mean(s, c->b, c->stream);
    }
    if (e == hipSuccess) e = launch_ctl_begin(c->b, 0, 0, 0.0, 1, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        rs = fail(CAVI_E_HIP, "create: %s", hipGetErrorString(e));
        cavi_destroy(c);
        return rs;
    }
    *out = c;
    return CAVI_OK;
}

cavi_status cavi_get_prior_mean(cavi_ctx *ctx, double *m0_host)
{
    if (!ctx || !m0_host) return fail(CAVI_E_INVAL, "NULL argument");
    HIPCHK(hipMemcpyAsync(m0_host, ctx->b.m0, sizeof(double) * ctx->s.G, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return CAVI_OK;
}

cavi_status cavi_set_state(cavi_ctx *ctx, const double *alpha, const double *m, const double *beta,
                           const double *a, const double *b)
{
    if (!ctx || !alpha || !m || !beta || !a || !b) return fail(CAVI_E_INVAL, "NULL argument");
    const int K = ctx->s.K, KG = K * ctx->s.G;
    for (int k = 0; k < K; ++k)
        if (!finite_pos(alpha[k])) return fail(CAVI_E_INVAL, "alpha[%d] must be finite and > 0", k);
    for (int i = 0; i < KG; ++i) {
        if (!isfinite(m[i])) return fail(CAVI_E_INVAL, "m[%d] is not finite", i);
        if (!finite_pos(beta[i]) || !finite_pos(a[i]) || !finite_pos(b[i]))
            return fail(CAVI_E_INVAL, "beta/a/b[%d] must be finite and > 0", i);
    }
    const Bufs &B = ctx->b;
    HIPCHK(hipMemcpyAsync(B.alpha, alpha, sizeof(double) * K, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(B.m, m, sizeof(double) * KG, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(B.beta, beta, sizeof(double) * KG, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(B.a, a, sizeof(double) * KG, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(B.b, b, sizeof(double) * KG, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(launch_coef(ctx->s, B, ctx->stream));
    HIPCHK(launch_ctl_begin(B, 0, 0, 0.0, 1, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->have_state = true;
    return CAVI_OK;
}

cavi_status cavi_get_state(cavi_ctx *ctx, double *alpha, double *m, double *beta, double *a, double *b)
{
    if (!ctx) return fail(CAVI_E_INVAL, "ctx is NULL");
    if (!ctx->have_state) return fail(CAVI_E_STATE, "no state: call cavi_init_standard or cavi_set_state");
    const int K = ctx->s.K, KG = K * ctx->s.G;
    const Bufs &B = ctx->b;
    if (alpha) HIPCHK(hipMemcpyAsync(alpha, B.alpha, sizeof(double) * K, hipMemcpyDeviceToHost, ctx->stream));
    if (m) HIPCHK(hipMemcpyAsync(m, B.m, sizeof(double) * KG, hipMemcpyDeviceToHost, ctx->stream));
    if (beta) HIPCHK(hipMemcpyAsync(beta, B.beta, sizeof(double) * KG, hipMemcpyDeviceToHost, ctx->stream));
    if (a) HIPCHK(hipMemcpyAsync(a, B.a, sizeof(double) * KG, hipMemcpyDeviceToHost, ctx->stream));
    if (b) HIPCHK(hipMemcpyAsync(b, B.b, sizeof(double) * KG, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return CAVI_OK;
}

// ---------------------------------------------------------------------------------------------
// standard initialisation (k-means++ with integer D^2 weights)

static cavi_status seed_row_to_device(cavi_ctx *c, int j, int64_t row)
{
    HIPCHK(hipMemcpyAsync(c->b.seeds + (size_t)j * c->s.G, c->b.x + (size_t)row * c->s.G, sizeof(float) * c->s.G,
                          hipMemcpyDeviceToDevice, c->stream));
    return CAVI_OK;
}

cavi_status cavi_init_standard(cavi_ctx *ctx, uint64_t seed)
{
    if (!ctx) return fail(CAVI_E_INVAL, "ctx is NULL");
    const Shape &s = ctx->s;
    const Bufs &B = ctx->b;
    hipStream_t st = ctx->stream;
    uint64_t rng = seed;
    int clog2n = 0;
    while (((int64_t)1 << clog2n) < s.N) ++clog2n;
    std::vector<double> bmax(s.nblk), blockd(kBlock);
    std::vector<unsigned long long> bsum(s.nblk);

    int64_t row = (int64_t)scaled_draw(rng, (uint64_t)s.N);
    cavi_status rs = seed_row_to_device(ctx, 0, row);
    if (rs != CAVI_OK) return rs;
    HIPCHK(launch_d2(s, B, 0, 1, st));
    for (int j = 1; j < s.K; ++j) {
        HIPCHK(hipMemcpyAsync(bmax.data(), B.blockmax, sizeof(double) * s.nblk, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        double mx = 0.0;
        for (int i = 0; i < s.nblk; ++i)
            if (bmax[i] > mx) mx = bmax[i];
        if (mx == 0.0) {
            row = (int64_t)scaled_draw(rng, (uint64_t)s.N);
        } else {
            int E;
            frexp(mx, &E);
            const int e = 62 - E - clog2n;
            HIPCHK(launch_wsum(s, B, e, st));
            HIPCHK(hipMemcpyAsync(bsum.data(), B.blocksum, sizeof(unsigned long long) * s.nblk,
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            unsigned long long W = 0;
            for (int i = 0; i < s.nblk; ++i) W += bsum[i];
            const uint64_t t = scaled_draw(rng, W);
            unsigned long long cum = 0;
            int blk = s.nblk - 1;
            for (int i = 0; i < s.nblk; ++i) {
                if (cum + bsum[i] > t) {
                    blk = i;
                    break;
                }
                cum += bsum[i];
            }
            const int64_t base = (int64_t)blk * kBlock;
            const int cnt = (int)std::min<int64_t>(kBlock, s.N - base);
            HIPCHK(hipMemcpyAsync(blockd.data(), B.mind2 + base, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            row = base + cnt - 1;
            for (int i = 0; i < cnt; ++i) {
                cum += (unsigned long long)floor(ldexp(blockd[i], e));
                if (cum > t) {
                    row = base + i;
                    break;
                }
            }
        }
        rs = seed_row_to_device(ctx, j, row);
        if (rs != CAVI_OK) return rs;
        HIPCHK(launch_d2(s, B, j, 0, st));
    }
    // statistics of the hard assignment are taken around the seed rows
    HIPCHK(hipMemcpyAsync(B.mf, B.seeds, sizeof(float) * s.K * s.G, hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_estep_stats(s, B, 1, st));
    HIPCHK(launch_reduce(s, B, 1, st));
    HIPCHK(launch_mstep(s, B, ctx->p, 1, st));
    HIPCHK(hipMemcpyAsync(ctx->hctl, B.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (ctx->hctl->numeric) return fail(CAVI_E_NUMERIC, "initial update produced a non-finite value");
    ctx->have_state = true;
    return CAVI_OK;
}

// ---------------------------------------------------------------------------------------------
// sweeps

static cavi_status enqueue_sweeps(cavi_ctx *c, int n)
{
    for (int i = 0; i < n; ++i) {
        HIPCHK(launch_estep_stats(c->s, c->b, 0, c->stream));
        HIPCHK(launch_reduce(c->s, c->b, 0, c->stream));
        HIPCHK(launch_mstep(c->s, c->b, c->p, 0, c->stream));
    }
    return CAVI_OK;
}

static cavi_status ensure_graph(cavi_ctx *c)
{
    if (c->graph) return CAVI_OK;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    cavi_status rs = enqueue_sweeps(c, kGraphSweeps);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rs != CAVI_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rs;
    }
    if (e != hipSuccess) return fail(CAVI_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->graph = nullptr;
        return fail(CAVI_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return CAVI_OK;
}

// Enqueue enough captured sweeps to cover n (the kernels skip past the call's limit).
static cavi_status replay(cavi_ctx *c, int n)
{
    cavi_status rs = ensure_graph(c);
    if (rs != CAVI_OK) return rs;
    for (int done = 0; done < n; done += kGraphSweeps) HIPCHK(hipGraphLaunch(c->graph, c->stream));
    return CAVI_OK;
}

cavi_status cavi_sweep(cavi_ctx *ctx, int32_t n, double *elbo_host)
{
    if (!ctx) return fail(CAVI_E_INVAL, "ctx is NULL");
    if (n < 0) return fail(CAVI_E_INVAL, "n=%d < 0", n);
    if (!ctx->have_state) return fail(CAVI_E_STATE, "no state: call cavi_init_standard or cavi_set_state");
    int done = 0;
    while (done < n) {
        const int seg = std::min(n - done, kHist);
        HIPCHK(launch_ctl_begin(ctx->b, seg, 0, 0.0, 0, ctx->stream));
        cavi_status rs = replay(ctx, seg);
        if (rs != CAVI_OK) return rs;
        if (elbo_host)
            HIPCHK(hipMemcpyAsync(elbo_host + done, ctx->b.hist, sizeof(double) * seg, hipMemcpyDeviceToHost,
                                  ctx->stream));
        HIPCHK(hipMemcpyAsync(ctx->hctl, ctx->b.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (ctx->hctl->numeric) {
            // the rejected update wrote coefficients; rebuild them from the kept state
            HIPCHK(launch_coef(ctx->s, ctx->b, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
            return fail(CAVI_E_NUMERIC, "sweep %d produced a non-finite value; state kept at sweep %d",
                        done + ctx->hctl->call_sweeps + 1, done + ctx->hctl->call_sweeps);
        }
        done += seg;
    }
    return CAVI_OK;
}

cavi_status cavi_run(cavi_ctx *ctx, int32_t max_sweeps, double rel_tol, int32_t *sweeps, double *elbo)
{
    if (!ctx) return fail(CAVI_E_INVAL, "ctx is NULL");
    if (max_sweeps < 1) return fail(CAVI_E_INVAL, "max_sweeps=%d < 1", max_sweeps);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol)) return fail(CAVI_E_INVAL, "rel_tol must be finite and >= 0");
    if (!ctx->have_state) return fail(CAVI_E_STATE, "no state: call cavi_init_standard or cavi_set_state");
    HIPCHK(launch_ctl_begin(ctx->b, max_sweeps, 1, rel_tol, 0, ctx->stream));
    int issued = 0;
    int batch = 1;  // graphs between host checks, doubled up to 4
    for (;;) {
        for (int i = 0; i < batch && issued < max_sweeps; ++i) {
            cavi_status rs = replay(ctx, kGraphSweeps);
            if (rs != CAVI_OK) return rs;
            issued += kGraphSweeps;
        }
        HIPCHK(hipMemcpyAsync(ctx->hctl, ctx->b.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        const Ctl &h = *ctx->hctl;
        if (h.numeric || h.converged || h.call_sweeps >= max_sweeps || issued >= max_sweeps) break;
        if (batch < 4) batch *= 2;
    }
    const Ctl &h = *ctx->hctl;
    if (sweeps) *sweeps = h.call_sweeps;
    if (elbo) *elbo = h.elbo;
    if (h.numeric) {
        HIPCHK(launch_coef(ctx->s, ctx->b, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        return fail(CAVI_E_NUMERIC, "sweep %d produced a non-finite value; state kept at sweep %d",
                    h.call_sweeps + 1, h.call_sweeps);
    }
    if (!h.converged) return fail(CAVI_E_NOTCONV, "not converged after %d sweeps", h.call_sweeps);
    return CAVI_OK;
}

cavi_status cavi_profile_estep(cavi_ctx *ctx, int32_t reps, float *avg_ms)
{
    if (!ctx || !avg_ms) return fail(CAVI_E_INVAL, "NULL argument");
    if (reps < 1) return fail(CAVI_E_INVAL, "reps=%d < 1", reps);
    if (!ctx->have_state) return fail(CAVI_E_STATE, "no state: call cavi_init_standard or cavi_set_state");
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(launch_ctl_begin(ctx->b, 1, 0, 0.0, 0, ctx->stream));
    HIPCHK(hipEventRecord(e0, ctx->stream));
    for (int i = 0; i < reps; ++i) HIPCHK(launch_estep_stats(ctx->s, ctx->b, 0, ctx->stream));
    HIPCHK(hipEventRecord(e1, ctx->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(launch_ctl_begin(ctx->b, 0, 0, 0.0, 0, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *avg_ms = ms / (float)reps;
    return CAVI_OK;
}

cavi_status cavi_get_responsibilities(cavi_ctx *ctx, float *r_dev)
{
    if (!ctx || !r_dev) return fail(CAVI_E_INVAL, "NULL argument");
    if (!ctx->have_state) return fail(CAVI_E_STATE, "no state: call cavi_init_standard or cavi_set_state");
    HIPCHK(launch_resp(ctx->s, ctx->b, r_dev, ctx->stream));
    return CAVI_OK;
}

}  // extern "C"
