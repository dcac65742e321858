// The entry point that allocates nothing: cavi_fit_static (include/cavi.h).  One dataset,
// standard initialisation, sweeps to convergence and the state copied out, with every device
// buffer carved from one static device array of kStaticBytes per GPU instead of a workspace.
// It enqueues the same kernels, in the same order, as cavi_create + cavi_init_standard +
// cavi_run + cavi_get_state, so the results are bitwise those of the handle path; only the
// launches differ (enqueued one by one instead of replayed from captured graphs).
#include <hip/hip_runtime.h>

#include <math.h>
#include <mutex>

#include "cavi_host.h"
#include "cavi_impl.h"

namespace cavi {

namespace {

constexpr size_t kStaticBytes = (size_t)64 << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;
constexpr int kCheckSweeps = 16;  // sweeps enqueued between convergence checks

// The device buffers of cavi_fit_static.  In host code this name is not a device address: the
// per-device address comes from hipGetSymbolAddress (scratch_ptr below).
__device__ __align__(256) unsigned char scratch[kStaticBytes];

// The one-dataset table and chunk map (every chunk belongs to dataset 0), written on the device
// so that nothing is staged from host memory.
__global__ void k_static_table(Ds d, Ds *ds, int32_t *chunk_ds, int nchunk)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) ds[0] = d;
    if (i < nchunk) chunk_ds[i] = 0;
}

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Address of this device's copy of the scratch array, looked up once per device with that
// device current.
cavi_status scratch_ptr(void **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CAVI_E_INVAL, "device %d is beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CAVI_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return CAVI_OK;
}

cavi_status sweeps_enqueue(const Shape &s, const Bufs &b, const Prior &p, int n, hipStream_t st)
{
    for (int i = 0; i < n; ++i) {
        HIPCHK(launch_estep_stats(s, b, 0, st));
        HIPCHK(launch_reduce(s, b, 0, st));
        HIPCHK(launch_mstep(s, b, p, 0, st));
    }
    return CAVI_OK;
}

}  // namespace

}  // namespace cavi

using namespace cavi;

extern "C" {

size_t cavi_static_scratch_bytes(void) { return kStaticBytes; }

cavi_status cavi_fit_static(const float *x_dev, int64_t N, int32_t G, int32_t K, const cavi_prior *prior,
                            uint64_t seed, int32_t max_sweeps, double rel_tol, void *hip_stream, double *alpha,
                            double *m, double *beta, double *a, double *b, int32_t *sweeps, double *elbo)
{
    if (!x_dev) return fail(CAVI_E_INVAL, "x_dev is NULL");
    if (((uintptr_t)x_dev) & 15) return fail(CAVI_E_INVAL, "x_dev is not 16-byte aligned");
    if (!alpha || !m || !beta || !a || !b) return fail(CAVI_E_INVAL, "NULL state array");
    if (max_sweeps < 1) return fail(CAVI_E_INVAL, "max_sweeps=%d < 1", max_sweeps);
    if (!(rel_tol >= 0.0) || !isfinite(rel_tol)) return fail(CAVI_E_INVAL, "rel_tol must be finite and >= 0");
    Shape s{};
    cavi_status rs = make_shape(1, &N, &K, G, kHistSingle, s, nullptr);
    if (rs != CAVI_OK) return rs;
    Prior p{};
    rs = check_prior(prior, p);
    if (rs != CAVI_OK) return rs;
    const bool have_m0 = prior && prior->m0;
    if (have_m0)
        for (int g = 0; g < G; ++g)
            if (!isfinite(prior->m0[g])) return fail(CAVI_E_INVAL, "prior m0[%d] is not finite", g);
    const size_t need = workspace_bytes(s);
    if (need > kStaticBytes)
        return fail(CAVI_E_NOMEM, "N=%lld, G=%d, K=%d needs %zu bytes of scratch; the static array holds %zu",
                    (long long)N, G, K, need, kStaticBytes);
    HIPCHK(prepare_kernels());
    s.tile_rows = choose_tile_rows(G, s.kt);
    if (s.tile_rows < 16) return fail(CAVI_E_INVAL, "G=%d needs more LDS per block than the device has", G);
    // the register-light E-step schedule where the tile leaves room for more waves (K > 8), else the
    // register-heavy one; both give bitwise the same results
    s.schedule = s.kt > 8 ? 1 : 0;
    void *ws = nullptr;
    rs = scratch_ptr(&ws);
    if (rs != CAVI_OK) return rs;
    hipStream_t st = (hipStream_t)hip_stream;
    Bufs bf{};
    carve(s, ws, bf);
    bf.x = x_dev;
    const Ds d{0, (int32_t)N, K, 0, s.nchunk};
    hipLaunchKernelGGL(k_static_table, dim3((s.nchunk + 255) / 256), dim3(256), 0, st, d, (Ds *)bf.ds,
                       (int32_t *)bf.chunk_ds, s.nchunk);
    HIPCHK(hipGetLastError());
    if (have_m0)
        HIPCHK(hipMemcpyAsync(bf.m0, prior->m0, sizeof(double) * G, hipMemcpyHostToDevice, st));
    else
        HIPCHK(launch_prior_mean(s, bf, st));
    HIPCHK(launch_ctl_begin(s, bf, 0, 0, 0.0, 1, st));
    // standard initialisation: k-means++ seeds, hard nearest-seed statistics, one update
    HIPCHK(launch_kmeanspp(s, bf, (unsigned long long)seed, st));
    HIPCHK(hipMemcpyAsync(bf.mf, bf.seeds, sizeof(float) * s.Kmax * G, hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_estep_stats(s, bf, 1, st));
    HIPCHK(launch_reduce(s, bf, 1, st));
    HIPCHK(launch_mstep(s, bf, p, 1, st));
    Ctl c{};
    HIPCHK(hipMemcpyAsync(&c, bf.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (c.numeric) return fail(CAVI_E_NUMERIC, "initial update is not finite");
    // sweeps until converged: a check after 16 sweeps, then every 32, as the handle's run
    HIPCHK(launch_ctl_begin(s, bf, max_sweeps, 1, rel_tol, 0, st));
    int issued = 0, batch = 1;
    for (;;) {
        for (int i = 0; i < batch && issued < max_sweeps; ++i) {
            rs = sweeps_enqueue(s, bf, p, kCheckSweeps, st);
            if (rs != CAVI_OK) return rs;
            issued += kCheckSweeps;
        }
        HIPCHK(launch_count_active(s, bf, st));
        int32_t active = 0;
        HIPCHK(hipMemcpyAsync(&active, bf.count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (active == 0 || issued >= max_sweeps) break;
        if (batch < 2) batch *= 2;
    }
    const size_t KG = (size_t)K * G;
    HIPCHK(hipMemcpyAsync(&c, bf.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(alpha, bf.alpha, sizeof(double) * K, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(m, bf.m, sizeof(double) * KG, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(beta, bf.beta, sizeof(double) * KG, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(a, bf.a, sizeof(double) * KG, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(b, bf.b, sizeof(double) * KG, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (sweeps) *sweeps = c.call_sweeps;
    if (elbo) *elbo = c.elbo;
    if (c.numeric)
        return fail(CAVI_E_NUMERIC, "sweep %d produced a non-finite value; state kept at sweep %d", c.sweeps + 1,
                    c.sweeps);
    if (!c.converged) return fail(CAVI_E_NOTCONV, "not converged after %d sweeps", max_sweeps);
    return CAVI_OK;
}

}  // extern "C"
