// Host runtime behind include/cavi.h: argument checks, workspace, the
// k-means++ initialisation drivers, hipGraph-captured sweeps and the
// convergence loops.  A single-dataset handle and a batch handle share one
// implementation (a single dataset is a batch of one).  All device work is in
// the .hip files.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/cavi.h"
#include "cavi_host.h"
#include "cavi_impl.h"

using namespace cavi;

namespace {

thread_local std::string g_err;

}  // namespace

namespace cavi {

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

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

constexpr int64_t kBatchChunkGrid = 2048;  // E-step workgroups of a batch launch

cavi_status make_shape(int32_t B, const int64_t *N, const int32_t *K, int32_t G, int hist_cap, Shape &s,
                       std::vector<Ds> *ds)
{
    if (B < 1) return fail(CAVI_E_INVAL, "B=%d < 1", B);
    if (G < 1 || G > kMaxG) return fail(CAVI_E_INVAL, "G=%d outside [1, %d]", G, kMaxG);
    int kmax = 0;
    int64_t ntot = 0, nmax = 0, nchunk = 0;
    for (int i = 0; i < B; ++i) {
        if (K[i] < 1 || K[i] > kMaxK) return fail(CAVI_E_INVAL, "K=%d outside [1, %d] (dataset %d)", K[i], kMaxK, i);
        if ((int64_t)K[i] * G > kMaxKG)
            return fail(CAVI_E_INVAL, "K*G=%lld exceeds %d (dataset %d)", (long long)K[i] * G, kMaxKG, i);
        if (N[i] < K[i]) return fail(CAVI_E_INVAL, "N=%lld < K=%d (dataset %d)", (long long)N[i], K[i], i);
        if (N[i] >= ((int64_t)1 << 31)) return fail(CAVI_E_INVAL, "N=%lld too large (dataset %d)", (long long)N[i], i);
        kmax = std::max(kmax, (int)K[i]);
        if (ds) ds->push_back(Ds{ntot, (int32_t)N[i], K[i], (int32_t)nchunk, (int32_t)((N[i] + kChunkRows - 1) / kChunkRows)});
        ntot += N[i];
        nmax = std::max(nmax, N[i]);
        nchunk += (N[i] + kChunkRows - 1) / kChunkRows;
    }
    if (nchunk >= ((int64_t)1 << 31)) return fail(CAVI_E_INVAL, "too many rows");
    s.B = B;
    s.G = G;
    s.Kmax = kmax;
    s.kt = choose_kt(kmax);
    s.Smax = kmax + 2 * kmax * G + 1;
    s.nchunk = (int32_t)nchunk;
    s.tile_rows = choose_tile_rows(G, s.kt);
    s.hist_cap = hist_cap;
    // batches: capped grids that loop over the work lists (a single dataset: one workgroup per chunk)
    s.egrid = B > 1 ? (int32_t)std::min<int64_t>(nchunk, kBatchChunkGrid) : (int32_t)nchunk;
    s.Ntot = ntot;
    s.Nmax = nmax;
    return CAVI_OK;
}

cavi_status check_prior(const cavi_prior *prior, Prior &p)
{
    cavi_prior pr;
    cavi_prior_default(&pr);
    if (prior) pr = *prior;
    if (!finite_pos(pr.alpha0) || !finite_pos(pr.beta0) || !finite_pos(pr.a0) || !finite_pos(pr.b0))
        return fail(CAVI_E_INVAL, "prior hyperparameters must be finite and > 0");
    p = Prior{pr.alpha0, pr.beta0, pr.a0, pr.b0};
    return CAVI_OK;
}


}  // namespace cavi

namespace {

constexpr int kGraphSweeps = 16;  // sweeps per captured graph (the largest of kGraphSizes)
constexpr int kGraphSizes[] = {16, 8, 4, 2, 1};  // a call of n sweeps replays n's binary digits
constexpr int kNumGraphs = sizeof(kGraphSizes) / sizeof(kGraphSizes[0]);
constexpr int kTuneChunks = 2048; // the autotuner times the E-step on at most this many chunks

struct Handle {
    Shape s{};
    Bufs b{};
    Prior p{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *ws = nullptr;
    bool own_ws = false;
    std::vector<Ds> ds;
    std::vector<char> have_state;
    bool coef_dirty = false;
    hipGraphExec_t graph[kNumGraphs] = {};  // kGraphSizes[i] sweeps each, captured on first use
    Ctl *hctl = nullptr;        // pinned host mirror of the control blocks
    int32_t *hcount = nullptr;  // pinned
    bool tuned = false;         // E-step schedule chosen (autotuned or set)
    float sched_ms[2] = {0.f, 0.f};
};

void destroy_handle(Handle *h)
{
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (hipGraphExec_t g : h->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    if (h->hctl) (void)hipHostFree(h->hctl);
    if (h->hcount) (void)hipHostFree(h->hcount);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

// Shared create: validation done by the caller except for device resources.
cavi_status create_handle(Handle *h, const float *x_dev, int32_t B, const int64_t *N, const int32_t *K, int32_t G,
                          const cavi_prior *prior, const double *m0_host, int hist_cap, void *hip_stream,
                          void *workspace_dev, size_t ws_bytes)
{
    if (!x_dev) return fail(CAVI_E_INVAL, "x_dev is NULL");
    if (((uintptr_t)x_dev) & 15) return fail(CAVI_E_INVAL, "x_dev is not 16-byte aligned");
    cavi_status st = make_shape(B, N, K, G, hist_cap, h->s, &h->ds);
    if (st != CAVI_OK) return st;
    st = check_prior(prior, h->p);
    if (st != CAVI_OK) return st;
    if (m0_host)
        for (size_t i = 0; i < (size_t)B * G; ++i)
            if (!isfinite(m0_host[i])) return fail(CAVI_E_INVAL, "prior m0[%zu] is not finite", i);
    const size_t need = workspace_bytes(h->s);
    if (workspace_dev) {
        if (ws_bytes < need) return fail(CAVI_E_NOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
        if (((uintptr_t)workspace_dev) & 255) return fail(CAVI_E_INVAL, "workspace is not 256-byte aligned");
    }
    hipError_t e = prepare_kernels();
    if (e != hipSuccess) return fail(CAVI_E_HIP, "device query: %s", hipGetErrorString(e));
    h->s.tile_rows = choose_tile_rows(G, h->s.kt);
    if (h->s.tile_rows < 16) return fail(CAVI_E_INVAL, "G=%d needs more LDS per block than the device has", G);
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreate(&h->stream);
        if (e != hipSuccess) return fail(CAVI_E_HIP, "hipStreamCreate: %s", hipGetErrorString(e));
        h->own_stream = true;
    }
    if (workspace_dev) {
        h->ws = workspace_dev;
    } else {
        e = hipMalloc(&h->ws, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->ws = nullptr;
            return fail(CAVI_E_NOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
        }
        h->own_ws = true;
    }
    HIPCHK(hipHostMalloc((void **)&h->hctl, sizeof(Ctl) * B, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&h->hcount, sizeof(int32_t), hipHostMallocDefault));
    carve(h->s, h->ws, h->b);
    h->b.x = x_dev;
    std::vector<int32_t> chunk_ds(h->s.nchunk);
    for (int i = 0; i < B; ++i)
        for (int c = 0; c < h->ds[i].nchunk; ++c) chunk_ds[h->ds[i].chunk0 + c] = i;
    HIPCHK(hipMemcpyAsync((void *)h->b.ds, h->ds.data(), sizeof(Ds) * B, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync((void *)h->b.chunk_ds, chunk_ds.data(), sizeof(int32_t) * h->s.nchunk,
                          hipMemcpyHostToDevice, h->stream));
    if (m0_host)
        HIPCHK(hipMemcpyAsync(h->b.m0, m0_host, sizeof(double) * B * G, hipMemcpyHostToDevice, h->stream));
    else
        HIPCHK(launch_prior_mean(h->s, h->b, h->stream));
    HIPCHK(launch_ctl_begin(h->s, h->b, 0, 0, 0.0, 1, h->stream));
    HIPCHK(launch_list_all(h->s, h->b, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->have_state.assign(B, 0);
    return CAVI_OK;
}

bool all_have_state(const Handle *h)
{
    for (char c : h->have_state)
        if (!c) return false;
    return true;
}

cavi_status set_state_one(Handle *h, int bi, const double *alpha, const double *m, const double *beta,
                          const double *a, const double *b)
{
    if (!alpha || !m || !beta || !a || !b) return fail(CAVI_E_INVAL, "NULL argument");
    const int K = h->ds[bi].K, G = h->s.G, KG = K * G;
    for (int k = 0; k < K; ++k)
        if (!finite_pos(alpha[k])) return fail(CAVI_E_INVAL, "alpha[%d] must be finite and > 0", k);
    for (int i = 0; i < KG; ++i) {
        if (!isfinite(m[i])) return fail(CAVI_E_INVAL, "m[%d] is not finite", i);
        if (!finite_pos(beta[i]) || !finite_pos(a[i]) || !finite_pos(b[i]))
            return fail(CAVI_E_INVAL, "beta/a/b[%d] must be finite and > 0", i);
    }
    const size_t kb = (size_t)bi * h->s.Kmax, kg = kb * G;
    const Bufs &B = h->b;
    HIPCHK(hipMemcpyAsync(B.alpha + kb, alpha, sizeof(double) * K, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(B.m + kg, m, sizeof(double) * KG, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(B.beta + kg, beta, sizeof(double) * KG, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(B.a + kg, a, sizeof(double) * KG, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(B.b + kg, b, sizeof(double) * KG, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->have_state[bi] = 1;
    h->coef_dirty = true;
    return CAVI_OK;
}

cavi_status refresh_coef(Handle *h)
{
    if (!h->coef_dirty) return CAVI_OK;
    HIPCHK(launch_coef(h->s, h->b, h->stream));
    HIPCHK(launch_ctl_begin(h->s, h->b, 0, 0, 0.0, 1, h->stream));
    h->coef_dirty = false;
    return CAVI_OK;
}

cavi_status get_state_one(Handle *h, int bi, double *alpha, double *m, double *beta, double *a, double *b)
{
    if (!h->have_state[bi]) return fail(CAVI_E_STATE, "no state: call init_standard or set_state");
    const int K = h->ds[bi].K, KG = K * h->s.G;
    const size_t kb = (size_t)bi * h->s.Kmax, kg = kb * h->s.G;
    const Bufs &B = h->b;
    if (alpha) HIPCHK(hipMemcpyAsync(alpha, B.alpha + kb, sizeof(double) * K, hipMemcpyDeviceToHost, h->stream));
    if (m) HIPCHK(hipMemcpyAsync(m, B.m + kg, sizeof(double) * KG, hipMemcpyDeviceToHost, h->stream));
    if (beta) HIPCHK(hipMemcpyAsync(beta, B.beta + kg, sizeof(double) * KG, hipMemcpyDeviceToHost, h->stream));
    if (a) HIPCHK(hipMemcpyAsync(a, B.a + kg, sizeof(double) * KG, hipMemcpyDeviceToHost, h->stream));
    if (b) HIPCHK(hipMemcpyAsync(b, B.b + kg, sizeof(double) * KG, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return CAVI_OK;
}

// statistics of the hard nearest-seed assignment, then one update, for every dataset
cavi_status finish_init(Handle *h)
{
    const Shape &s = h->s;
    const Bufs &B = h->b;
    HIPCHK(hipMemcpyAsync(B.mf, B.seeds, sizeof(float) * s.B * s.Kmax * s.G, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(launch_list_all(s, B, h->stream));
    HIPCHK(launch_estep_stats(s, B, 1, h->stream));
    HIPCHK(launch_reduce(s, B, 1, h->stream));
    HIPCHK(launch_mstep(s, B, h->p, 1, h->stream));
    HIPCHK(hipMemcpyAsync(h->hctl, B.ctl, sizeof(Ctl) * s.B, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int i = 0; i < s.B; ++i)
        if (h->hctl[i].numeric) return fail(CAVI_E_NUMERIC, "initial update of dataset %d is not finite", i);
    std::fill(h->have_state.begin(), h->have_state.end(), 1);
    h->coef_dirty = false;
    return CAVI_OK;
}

// standard initialisation of every dataset: k-means++ seeds on the device (dataset b uses the
// SplitMix64 state seed + b), hard nearest-seed statistics, one update
cavi_status init_all(Handle *h, uint64_t seed)
{
    HIPCHK(launch_kmeanspp(h->s, h->b, (unsigned long long)seed, h->stream));
    return finish_init(h);
}

cavi_status enqueue_sweeps(Handle *c, int n)
{
    for (int i = 0; i < n; ++i) {
        HIPCHK(launch_estep_stats(c->s, c->b, 0, c->stream));
        HIPCHK(launch_reduce(c->s, c->b, 0, c->stream));
        HIPCHK(launch_mstep(c->s, c->b, c->p, 0, c->stream));
        if (c->s.B > 1) HIPCHK(launch_compact(c->s, c->b, c->stream));
    }
    return CAVI_OK;
}

// Average duration (ms) of reps E-step launches with the handle's current schedule.  The
// E-step writes only the chunk partials, which the next sweep overwrites.
cavi_status time_estep(Handle *h, int reps, float *ms, int max_chunks = 0)
{
    Shape sh = h->s;
    if (max_chunks > 0 && sh.nchunk > max_chunks) sh.nchunk = max_chunks;
    sh.egrid = std::min(sh.egrid, sh.nchunk);
    HIPCHK(launch_list_all(h->s, h->b, h->stream));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(launch_ctl_begin(h->s, h->b, 1, 0, 0.0, 0, h->stream));
    HIPCHK(hipEventRecord(e0, h->stream));
    for (int i = 0; i < reps; ++i) HIPCHK(launch_estep_stats(sh, h->b, 0, h->stream));
    HIPCHK(hipEventRecord(e1, h->stream));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(launch_ctl_begin(h->s, h->b, 0, 0, 0.0, 0, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    *ms = t / (float)reps;
    return CAVI_OK;
}

// Autotuner: the tiled E-step has two schedules with identical results (register-heavy:
// unrolled exact terms, centres and responsibilities in registers; register-light: the same
// values kept in LDS, more waves per SIMD).  Which is faster depends on G, K and the LDS the
// tile takes, so both are timed on the handle's own data (its first kTuneChunks chunks, after
// one warm-up launch each) at the first sweep or run, before that call sets the control
// blocks and before the sweep graph is captured.
cavi_status autotune(Handle *h)
{
    if (h->tuned) return CAVI_OK;
    h->tuned = true;
    if (!tiled_supported(h->s.Kmax, h->s.G)) return CAVI_OK;
    float best = 0.f;
    int pick = 0;
    for (int v = 0; v < 2; ++v) {
        h->s.schedule = v;
        float warm = 0.f, t = 0.f;
        cavi_status rs = time_estep(h, 1, &warm, kTuneChunks);
        if (rs == CAVI_OK) rs = time_estep(h, 3, &t, kTuneChunks);
        if (rs != CAVI_OK) return rs;
        h->sched_ms[v] = t;
        if (v == 0 || t < best) {
            best = t;
            pick = v;
        }
    }
    h->s.schedule = pick;
    return CAVI_OK;
}

cavi_status ensure_graph(Handle *c, int gi)
{
    if (c->graph[gi]) return CAVI_OK;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    cavi_status rs = enqueue_sweeps(c, kGraphSizes[gi]);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rs != CAVI_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rs;
    }
    if (e != hipSuccess) return fail(CAVI_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph[gi], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->graph[gi] = nullptr;
        return fail(CAVI_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return CAVI_OK;
}

// Enqueue exactly n captured sweeps: 16-sweep graphs, then one graph per remaining binary digit
// of n (8, 4, 2, 1), so that a call never enqueues sweeps past its limit (the kernels would skip
// them, at the cost of their launches).
cavi_status replay(Handle *c, int n)
{
    for (int gi = 0; gi < kNumGraphs && n > 0; ++gi) {
        const int sz = kGraphSizes[gi];
        if (n < sz) continue;
        cavi_status rs = ensure_graph(c, gi);
        if (rs != CAVI_OK) return rs;
        const int reps = gi == 0 ? n / sz : 1;
        for (int r = 0; r < reps; ++r) HIPCHK(hipGraphLaunch(c->graph[gi], c->stream));
        n -= reps * sz;
    }
    return CAVI_OK;
}

cavi_status numeric_failure(Handle *h)
{
    // the rejected update wrote coefficients; rebuild them from the kept state
    HIPCHK(launch_coef(h->s, h->b, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int i = 0; i < h->s.B; ++i)
        if (h->hctl[i].numeric)
            return fail(CAVI_E_NUMERIC, "dataset %d: sweep %d produced a non-finite value; state kept at sweep %d", i,
                        h->hctl[i].sweeps + 1, h->hctl[i].sweeps);
    return fail(CAVI_E_NUMERIC, "non-finite value");
}

cavi_status sweep_n(Handle *h, int32_t n, double *elbo_host)
{
    if (n < 0) return fail(CAVI_E_INVAL, "n=%d < 0", n);
    if (!all_have_state(h)) return fail(CAVI_E_STATE, "no state: call init_standard or set_state");
    cavi_status rs = refresh_coef(h);
    if (rs == CAVI_OK) rs = autotune(h);  // before the control blocks are set for this call
    // every graph size is captured at the first call, so that no later call waits for a capture
    // (a few hundred microseconds of host work) before its first launch
    for (int gi = 0; gi < kNumGraphs && rs == CAVI_OK; ++gi) rs = ensure_graph(h, gi);
    if (rs != CAVI_OK) return rs;
    const int cap = h->s.hist_cap;
    int done = 0;
    while (done < n) {
        const int seg = std::min(n - done, elbo_host ? cap : n - done);
        HIPCHK(launch_ctl_begin(h->s, h->b, seg, 0, 0.0, 0, h->stream));
        HIPCHK(launch_list_all(h->s, h->b, h->stream));
        rs = replay(h, seg);
        if (rs != CAVI_OK) return rs;
        if (elbo_host)
            HIPCHK(hipMemcpyAsync(elbo_host + done, h->b.hist, sizeof(double) * seg, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(h->hctl, h->b.ctl, sizeof(Ctl) * h->s.B, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int i = 0; i < h->s.B; ++i)
            if (h->hctl[i].numeric) return numeric_failure(h);
        done += seg;
    }
    return CAVI_OK;
}

// returns CAVI_OK when every dataset converged, CAVI_E_NOTCONV otherwise
cavi_status run_all(Handle *h, int32_t max_sweeps, double rel_tol)
{
    if (max_sweeps < 1) return fail(CAVI_E_INVAL, "max_sweeps=%d < 1", max_sweeps);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol)) return fail(CAVI_E_INVAL, "rel_tol must be finite and >= 0");
    if (!all_have_state(h)) return fail(CAVI_E_STATE, "no state: call init_standard or set_state");
    cavi_status rs = refresh_coef(h);
    if (rs == CAVI_OK) rs = autotune(h);  // before the control blocks are set for this call
    if (rs != CAVI_OK) return rs;
    HIPCHK(launch_ctl_begin(h->s, h->b, max_sweeps, 1, rel_tol, 0, h->stream));
    HIPCHK(launch_list_all(h->s, h->b, h->stream));
    int issued = 0;
    // graphs between host checks: 1, then 2 (a check after 16 sweeps, then every 32).  Sweeps
    // enqueued after the last dataset has converged only skip, but each still costs its four
    // launches (about 19 us for a batch of 4,096 datasets): checking every 32 sweeps instead of
    // every 128 took such a batch's run (200 to 200,000 rows, G = 48) from 55.3 to 53.9 ms
    int batch = 1;
    for (;;) {
        for (int i = 0; i < batch && issued < max_sweeps; ++i) {
            rs = replay(h, kGraphSweeps);
            if (rs != CAVI_OK) return rs;
            issued += kGraphSweeps;
        }
        HIPCHK(launch_count_active(h->s, h->b, h->stream));
        HIPCHK(hipMemcpyAsync(h->hcount, h->b.count, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (*h->hcount == 0 || issued >= max_sweeps) break;
        if (batch < 2) batch *= 2;
    }
    HIPCHK(hipMemcpyAsync(h->hctl, h->b.ctl, sizeof(Ctl) * h->s.B, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    int notconv = 0;
    for (int i = 0; i < h->s.B; ++i) {
        if (h->hctl[i].numeric) return numeric_failure(h);
        if (!h->hctl[i].converged) ++notconv;
    }
    if (notconv) return fail(CAVI_E_NOTCONV, "%d dataset(s) not converged after %d sweeps", notconv, max_sweeps);
    return CAVI_OK;
}

}  // namespace

namespace cavi {
void set_last_error(const char *msg) { g_err = msg; }
}  // namespace cavi

struct cavi_ctx {
    Handle h;
};

struct cavi_batch {
    Handle h;
};

extern "C" {

const char *cavi_last_error(void) { return g_err.c_str(); }

const char *cavi_version(void) { return "cavi-gfx950 0.2.0"; }

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

// ---------------------------------------------------------------------------------------------
// single dataset

cavi_status cavi_workspace_bytes(int64_t N, int32_t G, int32_t K, size_t *bytes)
{
    if (!bytes) return fail(CAVI_E_INVAL, "bytes is NULL");
    Shape s;
    cavi_status st = make_shape(1, &N, &K, G, kHistSingle, s, nullptr);
    if (st != CAVI_OK) return st;
    *bytes = workspace_bytes(s);
    return CAVI_OK;
}

cavi_status cavi_create(cavi_ctx **out, const float *x_dev, int64_t N, int32_t G, int32_t K,
                        const cavi_prior *prior, void *hip_stream, void *workspace_dev, size_t ws_bytes)
{
    if (!out) return fail(CAVI_E_INVAL, "out is NULL");
    *out = nullptr;
    cavi_ctx *c = new cavi_ctx;
    cavi_status st = create_handle(&c->h, x_dev, 1, &N, &K, G, prior, prior ? prior->m0 : nullptr, kHistSingle,
                                   hip_stream, workspace_dev, ws_bytes);
    if (st != CAVI_OK) {
        destroy_handle(&c->h);
        delete c;
        return st;
    }
    *out = c;
    return CAVI_OK;
}

cavi_status cavi_destroy(cavi_ctx *ctx)
{
    if (!ctx) return CAVI_OK;
    destroy_handle(&ctx->h);
    delete ctx;
    return CAVI_OK;
}

cavi_status cavi_get_prior_mean(cavi_ctx *ctx, double *m0_host)
{
    if (!ctx || !m0_host) return fail(CAVI_E_INVAL, "NULL argument");
    HIPCHK(hipMemcpyAsync(m0_host, ctx->h.b.m0, sizeof(double) * ctx->h.s.G, hipMemcpyDeviceToHost, ctx->h.stream));
    HIPCHK(hipStreamSynchronize(ctx->h.stream));
    return CAVI_OK;
}

cavi_status cavi_init_standard(cavi_ctx *ctx, uint64_t seed)
{
    if (!ctx) return fail(CAVI_E_INVAL, "ctx is NULL");
    return init_all(&ctx->h, seed);
}

cavi_status cavi_set_state(cavi_ctx *ctx, const double *alpha, const double *m, const double *beta,
                           const double *a, const double *b)
{
    if (!ctx) return fail(CAVI_E_INVAL, "NULL argument");
    cavi_status st = set_state_one(&ctx->h, 0, alpha, m, beta, a, b);
    if (st != CAVI_OK) return st;
    st = refresh_coef(&ctx->h);
    if (st != CAVI_OK) return st;
    HIPCHK(hipStreamSynchronize(ctx->h.stream));
    return CAVI_OK;
}

cavi_status cavi_get_state(cavi_ctx *ctx, double *alpha, double *m, double *beta, double *a, double *b)
{
    if (!ctx) return fail(CAVI_E_INVAL, "ctx is NULL");
    return get_state_one(&ctx->h, 0, alpha, m, beta, a, b);
}

cavi_status cavi_sweep(cavi_ctx *ctx, int32_t n, double *elbo_host)
{
    if (!ctx) return fail(CAVI_E_INVAL, "ctx is NULL");
    return sweep_n(&ctx->h, n, elbo_host);
}

cavi_status cavi_run(cavi_ctx *ctx, int32_t max_sweeps, double rel_tol, int32_t *sweeps, double *elbo)
{
    if (!ctx) return fail(CAVI_E_INVAL, "ctx is NULL");
    cavi_status st = run_all(&ctx->h, max_sweeps, rel_tol);
    if (st == CAVI_OK || st == CAVI_E_NOTCONV) {
        if (sweeps) *sweeps = ctx->h.hctl[0].call_sweeps;
        if (elbo) *elbo = ctx->h.hctl[0].elbo;
    }
    return st;
}

cavi_status cavi_profile_estep(cavi_ctx *ctx, int32_t reps, float *avg_ms)
{
    if (!ctx || !avg_ms) return fail(CAVI_E_INVAL, "NULL argument");
    if (reps < 1) return fail(CAVI_E_INVAL, "reps=%d < 1", reps);
    Handle *h = &ctx->h;
    if (!all_have_state(h)) return fail(CAVI_E_STATE, "no state: call cavi_init_standard or cavi_set_state");
    cavi_status rs = refresh_coef(h);
    if (rs == CAVI_OK) rs = autotune(h);
    if (rs != CAVI_OK) return rs;
    return time_estep(h, reps, avg_ms);
}

cavi_status cavi_probe_read(const float *x_dev, int64_t n, float *out_dev, int32_t grid, int32_t reps,
                            void *hip_stream, float *avg_ms)
{
    if (!x_dev || !out_dev || !avg_ms) return fail(CAVI_E_INVAL, "NULL argument");
    if (n < 1 || grid < 1 || reps < 1) return fail(CAVI_E_INVAL, "n, grid and reps must be >= 1");
    if (((uintptr_t)x_dev) & 15) return fail(CAVI_E_INVAL, "x_dev is not 16-byte aligned");
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(launch_read_probe(x_dev, n, out_dev, grid, st));  // warm-up
    HIPCHK(hipEventRecord(e0, st));
    for (int i = 0; i < reps; ++i) HIPCHK(launch_read_probe(x_dev, n, out_dev, grid, st));
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = t / (float)reps;
    return CAVI_OK;
}

static cavi_status get_schedule(Handle *h, int32_t *schedule, float *ms)
{
    if (schedule) *schedule = h->s.schedule;
    if (ms) {
        ms[0] = h->sched_ms[0];
        ms[1] = h->sched_ms[1];
    }
    return CAVI_OK;
}

static cavi_status set_schedule(Handle *h, int32_t schedule)
{
    if (schedule < -1 || schedule > 2) return fail(CAVI_E_INVAL, "schedule=%d outside [-1, 2]", schedule);
    if (schedule == 2 && !(tiled_supported(h->s.Kmax, h->s.G) && h->s.kt == 16))
        return fail(CAVI_E_INVAL, "schedule 2 (the screen as a matrix product) needs G in {16, 32, 48, 64} and 9 to "
                                  "16 subpopulations");
    for (hipGraphExec_t &g : h->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    if (schedule == -1) {
        h->tuned = false;
        h->s.schedule = 0;
    } else {
        h->tuned = true;
        h->s.schedule = schedule;
    }
    return CAVI_OK;
}

cavi_status cavi_get_schedule(cavi_ctx *ctx, int32_t *schedule, float *ms)
{
    if (!ctx) return fail(CAVI_E_INVAL, "ctx is NULL");
    return get_schedule(&ctx->h, schedule, ms);
}

cavi_status cavi_set_schedule(cavi_ctx *ctx, int32_t schedule)
{
    if (!ctx) return fail(CAVI_E_INVAL, "ctx is NULL");
    return set_schedule(&ctx->h, schedule);
}

cavi_status cavi_batch_get_schedule(cavi_batch *bt, int32_t *schedule, float *ms)
{
    if (!bt) return fail(CAVI_E_INVAL, "batch is NULL");
    return get_schedule(&bt->h, schedule, ms);
}

cavi_status cavi_batch_set_schedule(cavi_batch *bt, int32_t schedule)
{
    if (!bt) return fail(CAVI_E_INVAL, "batch is NULL");
    return set_schedule(&bt->h, schedule);
}

cavi_status cavi_get_responsibilities(cavi_ctx *ctx, float *r_dev)
{
    if (!ctx || !r_dev) return fail(CAVI_E_INVAL, "NULL argument");
    if (!all_have_state(&ctx->h)) return fail(CAVI_E_STATE, "no state: call cavi_init_standard or cavi_set_state");
    cavi_status rs = refresh_coef(&ctx->h);
    if (rs != CAVI_OK) return rs;
    HIPCHK(launch_resp(ctx->h.s, ctx->h.b, r_dev, ctx->h.stream));
    return CAVI_OK;
}

// ---------------------------------------------------------------------------------------------
// batches

cavi_status cavi_batch_workspace_bytes(int32_t B, const int64_t *N, const int32_t *K, int32_t G, size_t *bytes)
{
    if (!bytes || !N || !K) return fail(CAVI_E_INVAL, "NULL argument");
    Shape s;
    cavi_status st = make_shape(B, N, K, G, 1, s, nullptr);
    if (st != CAVI_OK) return st;
    *bytes = workspace_bytes(s);
    return CAVI_OK;
}

cavi_status cavi_batch_create(cavi_batch **out, int32_t B, const float *x_dev, const int64_t *N, const int32_t *K,
                              int32_t G, const cavi_prior *prior, void *hip_stream, void *workspace_dev,
                              size_t ws_bytes)
{
    if (!out) return fail(CAVI_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!N || !K) return fail(CAVI_E_INVAL, "N or K is NULL");
    cavi_batch *c = new cavi_batch;
    cavi_status st = create_handle(&c->h, x_dev, B, N, K, G, prior, prior ? prior->m0 : nullptr, 1, hip_stream,
                                   workspace_dev, ws_bytes);
    if (st != CAVI_OK) {
        destroy_handle(&c->h);
        delete c;
        return st;
    }
    *out = c;
    return CAVI_OK;
}

cavi_status cavi_batch_destroy(cavi_batch *bt)
{
    if (!bt) return CAVI_OK;
    destroy_handle(&bt->h);
    delete bt;
    return CAVI_OK;
}

cavi_status cavi_batch_init_standard(cavi_batch *bt, uint64_t seed)
{
    if (!bt) return fail(CAVI_E_INVAL, "batch is NULL");
    return init_all(&bt->h, seed);
}

cavi_status cavi_batch_set_state(cavi_batch *bt, int32_t b, const double *alpha, const double *m,
                                 const double *beta, const double *a, const double *bb)
{
    if (!bt) return fail(CAVI_E_INVAL, "batch is NULL");
    if (b < 0 || b >= bt->h.s.B) return fail(CAVI_E_INVAL, "dataset %d outside [0, %d)", b, bt->h.s.B);
    return set_state_one(&bt->h, b, alpha, m, beta, a, bb);
}

cavi_status cavi_batch_set_state_warm(cavi_batch *bt, const float *out_dev, int32_t ld)
{
    if (!bt || !out_dev) return fail(CAVI_E_INVAL, "NULL argument");
    Handle *h = &bt->h;
    for (int i = 0; i < h->s.B; ++i) {
        const int64_t need = (int64_t)h->ds[i].K * (2 * h->s.G + 1);
        if (ld < need) return fail(CAVI_E_INVAL, "ld=%d < K(2G+1)=%lld (dataset %d)", ld, (long long)need, i);
    }
    HIPCHK(launch_warm_state(h->s, h->b, h->p, out_dev, ld, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    std::fill(h->have_state.begin(), h->have_state.end(), 1);
    h->coef_dirty = true;
    return CAVI_OK;
}

cavi_status cavi_batch_get_rows(cavi_batch *bt, float *rows_dev, int32_t ld, int32_t with_centre)
{
    if (!bt || !rows_dev) return fail(CAVI_E_INVAL, "NULL argument");
    Handle *h = &bt->h;
    if (!all_have_state(h)) return fail(CAVI_E_STATE, "no state: call init_standard or set_state");
    for (int i = 0; i < h->s.B; ++i) {
        const int64_t need = (int64_t)h->ds[i].K * (2 * h->s.G + 1) + (with_centre ? h->s.G : 0);
        if (ld < need) return fail(CAVI_E_INVAL, "ld=%d < %lld (dataset %d)", ld, (long long)need, i);
    }
    HIPCHK(launch_state_rows(h->s, h->b, h->p, rows_dev, ld, with_centre ? 1 : 0, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return CAVI_OK;
}

cavi_status cavi_batch_get_state(cavi_batch *bt, int32_t b, double *alpha, double *m, double *beta, double *a,
                                 double *bb)
{
    if (!bt) return fail(CAVI_E_INVAL, "batch is NULL");
    if (b < 0 || b >= bt->h.s.B) return fail(CAVI_E_INVAL, "dataset %d outside [0, %d)", b, bt->h.s.B);
    return get_state_one(&bt->h, b, alpha, m, beta, a, bb);
}

cavi_status cavi_batch_sweep(cavi_batch *bt, int32_t n)
{
    if (!bt) return fail(CAVI_E_INVAL, "batch is NULL");
    return sweep_n(&bt->h, n, nullptr);
}

cavi_status cavi_batch_run(cavi_batch *bt, int32_t max_sweeps, double rel_tol, int32_t *sweeps, double *elbo,
                           int32_t *n_converged)
{
    if (!bt) return fail(CAVI_E_INVAL, "batch is NULL");
    Handle *h = &bt->h;
    cavi_status st = run_all(h, max_sweeps, rel_tol);
    if (st == CAVI_OK || st == CAVI_E_NOTCONV) {
        int nc = 0;
        for (int i = 0; i < h->s.B; ++i) {
            if (sweeps) sweeps[i] = h->hctl[i].call_sweeps;
            if (elbo) elbo[i] = h->hctl[i].elbo;
            nc += h->hctl[i].converged ? 1 : 0;
        }
        if (n_converged) *n_converged = nc;
    }
    return st;
}

}  // extern "C"
