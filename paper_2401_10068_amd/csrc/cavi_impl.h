// Internal interface between the host runtime (cavi_api.cpp) and the gfx950
// kernels (cavi_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cavi {

// Rows per reduction chunk.  The sums over rows are defined as FP64 sums,
// in chunk order, of per-chunk partials; this constant is part of that
// definition (it fixes the bits), not a tuning knob.
constexpr int kChunkRows = 2048;
constexpr int kBlock = 256;
// Responsibilities below exp(-kLogRCut) of the row's normaliser are zero.
constexpr float kLogRCut = 87.0f;
// Bound history capacity on the device.
constexpr int kHist = 4096;
constexpr int kMaxK = 64;
constexpr int kMaxG = 512;
constexpr int kMaxKG = 4096;

// Control block in device memory (one per dataset).
struct Ctl {
    int32_t sweeps;        // sweeps since the state was set / initialised
    int32_t call_sweeps;   // sweeps of the current sweep/run call
    int32_t max_call;      // the current call runs at most this many sweeps
    int32_t stop_on_conv;  // 1: sweeps after convergence are no-ops
    int32_t converged;     // relative change test passed in this call
    int32_t numeric;       // a sweep produced a non-finite value (not committed)
    int32_t pad0, pad1;
    double tol;            // relative tolerance of the convergence test
    double elbo;           // bound after the last committed sweep
    double elbo_prev;      // bound one sweep earlier (same call)
};

struct Prior {
    double alpha0, beta0, a0, b0;
};

// Device buffers of one dataset (all carved from one workspace).
struct Bufs {
    const float *x;     // N x G data (caller-owned)
    double *alpha;      // K      state q(pi)
    double *m, *beta, *a, *b;  // K*G state q(mu, tau), k-major
    double *nalpha, *nm, *nbeta, *na, *nb;  // next-state staging
    double *m0;         // G prior centre
    double *tmp;        // K*G scratch
    float *cc;          // K   per-subpopulation constant of the row log-likelihood
    float *hq;          // 2*K*G interleaved (h, q): u = h x + q, l = c - sum u^2
    float *mf;          // K*G FP32 centre of the statistics (FP32 of m)
    float *seeds;       // K*G seed rows (initialisation)
    double *partials;   // nchunk * S per-chunk statistics
    double *totals;     // S
    double *hist;       // kHist bounds
    Ctl *ctl;
    double *mind2;      // N   (initialisation)
    double *blockmax;   // nblk
    unsigned long long *blocksum;  // nblk
    double *colpart;    // nchunk * G (prior centre)
};

struct Shape {
    int64_t N;
    int32_t G, K;
    int32_t nchunk;     // ceil(N / kChunkRows)
    int32_t S;          // K + 2 K G + 1 statistics per chunk
    int32_t tile_rows;  // rows staged in LDS per tile
    int32_t kt;         // compiled K bound (4, 8, 16, 32, 64)
    int32_t nblk;       // ceil(N / kBlock)
};

__device__ __forceinline__ bool sweep_skipped(const Ctl *c)
{
    return c->numeric || c->call_sweeps >= c->max_call || (c->stop_on_conv && c->converged);
}

// Bytes of LDS per block the device allows (set by prepare_kernels()).
extern int g_lds_limit;

size_t workspace_bytes(const Shape &s);
void carve(const Shape &s, void *ws, Bufs &b);
int choose_tile_rows(int G, int kt);
int choose_kt(int K);

// Once per process, before the first launch: kernel attributes (dynamic LDS limit).
hipError_t prepare_kernels();

// Launchers (enqueue only; return hipError_t of the launch).
hipError_t launch_estep_stats(const Shape &s, const Bufs &b, int init_mode, hipStream_t st);
// Tiled E-step kernel (estep_tiled.hip) for G in {16,32,48,64,96,128} and small K.
bool tiled_supported(int K, int G);
hipError_t launch_estep_tiled(const Shape &s, const Bufs &b, hipStream_t st);
hipError_t launch_reduce(const Shape &s, const Bufs &b, int init_mode, hipStream_t st);
hipError_t launch_mstep(const Shape &s, const Bufs &b, const Prior &p, int init_mode, hipStream_t st);
hipError_t launch_coef(const Shape &s, const Bufs &b, hipStream_t st);
hipError_t launch_prior_mean(const Shape &s, const Bufs &b, hipStream_t st);
hipError_t launch_d2(const Shape &s, const Bufs &b, int seed_index, int first, hipStream_t st);
hipError_t launch_wsum(const Shape &s, const Bufs &b, int e, hipStream_t st);
hipError_t launch_resp(const Shape &s, const Bufs &b, float *r, hipStream_t st);
hipError_t launch_ctl_begin(const Bufs &b, int max_call, int stop_on_conv, double tol, int reset,
                            hipStream_t st);

}  // namespace cavi
