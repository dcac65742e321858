// Internal interface between the host runtime (cavi_api.cpp) and the gfx950
// kernels.  Not part of the public ABI.
//
// Every handle is a batch of B datasets that share G (a single-dataset
// handle is a batch of one).  Rows of all datasets are concatenated in one
// FP32 array; each dataset's rows are cut into 2048-row chunks numbered
// globally.  Per-dataset arrays use a uniform stride of Kmax subpopulations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cavi {

// Rows per reduction chunk.  The sums over rows are defined as FP64 sums,
// in chunk order, of per-chunk partials; this constant is part of that
// definition (it fixes the bits), not a tuning knob.
constexpr int kChunkRows = 2048;
constexpr int kRedSplit = 4;          // chunk ranges of a large dataset
constexpr int kSplitMinChunks = 128;  // a dataset of at least this many chunks is large

// Chunk ranges a dataset of nchunk chunks is reduced in (the update adds their sums in order): 4 from
// 128 chunks up, else 1.  A function of the dataset alone, so that it sums the same way alone and in
// a batch.  (More ranges make the update's sums slower than the reduction gets faster.)
__host__ __device__ inline int red_split(int64_t nchunk) { return nchunk >= kSplitMinChunks ? kRedSplit : 1; }

// Ranges of the handle's largest dataset: the stride of the per-dataset range sums.
__host__ __device__ inline int red_split_max(int64_t Nmax) { return red_split((Nmax + kChunkRows - 1) / kChunkRows); }
constexpr int kBlock = 256;
// Responsibilities below exp(-kLogRCut) of the row's normaliser are zero.
constexpr float kLogRCut = 87.0f;
constexpr int kMaxK = 64;
constexpr int kMaxG = 512;
constexpr int kMaxKG = 4096;

// Control block in device memory, one per dataset.
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

// One dataset of a batch (device memory).
struct Ds {
    int64_t row0;     // first row in the concatenated data
    int32_t N, K;     // rows, subpopulations
    int32_t chunk0;   // first global chunk
    int32_t nchunk;   // chunks of this dataset
};

// nearest[] value of a row whose distance to seed 0 is NaN: the hard assignment takes seed 0
// whatever the later distances (the first-minimum scan keeps its first element when that is NaN)
constexpr uint8_t kNearestLocked = 255;

struct Shape {
    int32_t B;          // datasets
    int32_t G;          // genes (shared)
    int32_t Kmax;       // stride of the per-dataset subpopulation arrays
    int32_t kt;         // compiled K bound covering Kmax (4, 8, 16, 32, 64)
    int32_t Smax;       // statistics per chunk: Kmax + 2 Kmax G + 1
    int32_t nchunk;     // chunks of all datasets
    int32_t tile_rows;  // rows per LDS tile of the generic kernel
    int32_t hist_cap;   // bounds kept per dataset
    int32_t schedule;   // tiled E-step schedule: 0 register-heavy, 1 register-light (autotuned)
    int32_t egrid;      // workgroups of an E-step launch (batches: a capped grid over the work list)
    int64_t Ntot;       // rows of all datasets
    int64_t Nmax;       // rows of the largest dataset
};

// Device buffers (carved from one workspace, plus the caller's data).
struct Bufs {
    const float *x;       // Ntot x G data (caller-owned)
    const Ds *ds;         // B
    const int32_t *chunk_ds;  // nchunk: dataset of each global chunk
    double *alpha;        // B x Kmax          q(pi)
    double *m, *beta, *a, *b;  // B x Kmax x G  q(mu, tau)
    double *nm, *nbeta, *na, *nb;  // next-state staging (update items past the block size)
    double *m0;           // B x G prior centre
    float *cc;            // B x Kmax         c_k of the row log-likelihood
    float *hq;            // B x Kmax x G x 2  (h, q): u = h x + q, l = c - sum u^2
    float *mf;            // B x Kmax x G     FP32 centre of the statistics
    float *seeds;         // B x Kmax x G     seed rows (initialisation)
    double *partials;     // nchunk x Smax    per-chunk statistics
    double *totals;       // B x red_split_max(Nmax) x Smax: per dataset, the sums of its red_split(nchunk) chunk ranges
    double *hist;         // B x hist_cap     bound after each sweep
    Ctl *ctl;             // B
    int32_t *count;       // 1: datasets still sweeping
    double *mind2;        // Ntot             (initialisation)
    uint8_t *nearest;     // Ntot             (initialisation) nearest seed so far, kNearestLocked: seed 0
    double *blockmax;     // nchunk           (initialisation)
    unsigned long long *blocksum;  // nchunk  (initialisation)
    double *colpart;      // nchunk x G      (prior centre)
    int32_t *act_n;       // 2: datasets and chunks on the work lists (batches)
    int32_t *act_ds;      // B: datasets that still sweep, ascending
    int32_t *act_chunk;   // nchunk: their chunks, ascending
};

// Work lists of a batch: after every sweep the datasets that still sweep, and their chunks, are
// listed, so that the next sweep's launches (capped grids that loop over the lists) spend nothing
// on finished datasets.  A single-dataset handle takes its chunks directly.  Entries past a
// dataset's end of sweeping are skipped by sweep_skipped() as before, so a stale list is safe.
__device__ __forceinline__ int n_active_chunks(const Shape &s, const Bufs &b)
{
    return s.B == 1 ? s.nchunk : min(s.nchunk, b.act_n[1]);
}
__device__ __forceinline__ int active_chunk(const Shape &s, const Bufs &b, int i) { return s.B == 1 ? i : b.act_chunk[i]; }
__device__ __forceinline__ int n_active_datasets(const Shape &s, const Bufs &b) { return s.B == 1 ? 1 : min(s.B, b.act_n[0]); }
__device__ __forceinline__ int active_dataset(const Shape &s, const Bufs &b, int i) { return s.B == 1 ? 0 : b.act_ds[i]; }

// Record of dataset bi; a single-dataset handle's follows from the shape, without a load.
__device__ __forceinline__ Ds dataset(const Shape &s, const Bufs &b, int bi)
{
    return s.B == 1 ? Ds{0, (int32_t)s.Ntot, s.Kmax, 0, s.nchunk} : b.ds[bi];
}

__device__ __forceinline__ bool sweep_skipped(const Ctl *c)
{
    // every field loaded (no short-circuit), so that the loads overlap
    const int32_t cs = c->call_sweeps, mx = c->max_call, so = c->stop_on_conv, cv = c->converged, nu = c->numeric;
    return (nu != 0) | (cs >= mx) | ((so != 0) & (cv != 0));
}

// Text returned by cavi_last_error() for the calling thread.
void set_last_error(const char *msg);

// Bytes of LDS per block the device allows (set by prepare_kernels()).
extern int g_lds_limit;

size_t workspace_bytes(const Shape &s);
void carve(const Shape &s, void *ws, Bufs &b);
int choose_tile_rows(int G, int kt);
int choose_kt(int K);

// Once per process, before the first launch: kernel attributes (dynamic LDS limit).
hipError_t prepare_kernels();

// Launchers (enqueue only; return hipError_t of the launch).  init_mode: the
// hard nearest-seed responsibilities of the standard initialisation.
hipError_t launch_estep_stats(const Shape &s, const Bufs &b, int init_mode, hipStream_t st);
// Tiled E-step kernel (estep_tiled.hip) for G in {16,32,48,64,96,128} and small K.
bool tiled_supported(int K, int G);
hipError_t launch_estep_tiled(const Shape &s, const Bufs &b, int init_mode, hipStream_t st);
hipError_t launch_reduce(const Shape &s, const Bufs &b, int init_mode, hipStream_t st);
hipError_t launch_mstep(const Shape &s, const Bufs &b, const Prior &p, int init_mode, hipStream_t st);
hipError_t launch_coef(const Shape &s, const Bufs &b, hipStream_t st);
hipError_t launch_prior_mean(const Shape &s, const Bufs &b, hipStream_t st);
hipError_t launch_resp(const Shape &s, const Bufs &b, float *r, hipStream_t st);
hipError_t launch_ctl_begin(const Shape &s, const Bufs &b, int max_call, int stop_on_conv, double tol, int reset,
                            hipStream_t st);
hipError_t launch_count_active(const Shape &s, const Bufs &b, hipStream_t st);
// Work lists: every dataset and chunk (before a call's first sweep), or the datasets that still
// sweep and their chunks (after each sweep of a batch).
hipError_t launch_list_all(const Shape &s, const Bufs &b, hipStream_t st);
hipError_t launch_compact(const Shape &s, const Bufs &b, hipStream_t st);
// k-means++ seeds of every dataset (dataset b: SplitMix64 state seed + b), a few launches
// per seed and no host synchronisation; leaves the seeds in b.seeds.
hipError_t launch_kmeanspp(const Shape &s, const Bufs &b, unsigned long long seed, hipStream_t st);

// Plain streaming read of n floats from x (16-byte aligned) by grid workgroups; out receives grid
// per-workgroup sums.  The achievable-read reference of the roofline.
hipError_t launch_read_probe(const float *x, int64_t n, float *out, int grid, hipStream_t st);

// Learned warm start (warmstart.hip).
hipError_t launch_features(const float *x, const int64_t *row_off, int B, int G, float *feat, hipStream_t st);
hipError_t launch_features_quantiles(const float *x, const int64_t *row_off, int B, int G, float *feat, hipStream_t st);
hipError_t launch_targets(const double *pi, const double *mu, const double *tau, int B, int K, int G, float *tgt,
                          hipStream_t st);
hipError_t launch_gemm(bool ta, bool tb, int M, int N, int K, const float *A, int lda, const float *B, int ldb,
                       const float *bias, float *Z, float *Y, int ldc, int act, hipStream_t st);
hipError_t launch_gelu_back(int n, const float *Z, const float *dY, float *dZ, hipStream_t st);
hipError_t launch_colsum(int M, int N, const float *D, float *out, hipStream_t st);
hipError_t launch_mse(int n, float scale, const float *Y, const float *T, float *dY, double *part, hipStream_t st);
hipError_t launch_adamw(int64_t n, float *w, const float *g, float *m, float *v, float lr, float b1, float b2,
                        float eps, float wd, float c1, float c2, hipStream_t st);
hipError_t launch_warm_state(const Shape &s, const Bufs &b, const Prior &p, const float *out, int ld, hipStream_t st);
hipError_t launch_state_rows(const Shape &s, const Bufs &b, const Prior &p, float *rows, int ld, int centre,
                             hipStream_t st);
hipError_t launch_rows_axpy(int n, int m, float alpha, const float *x, int ldx, float *y, int ldy, hipStream_t st);

}  // namespace cavi
