// gfx950 kernels of the mixture CAVI sweep: the generic E-step + statistics
// kernel (any G, K up to 64; also the hard assignment of the standard
// initialisation), prior centres, control blocks, responsibilities, and the
// k-means++ seeding of the standard initialisation.
//
// One sweep (eq 12 applied to each factor of the mean-field family of eqs 9
// and 13, Section 3.4) is three launches over all datasets of a handle:
//   E-step + statistics  per 2048-row chunk (k_estep_stats here, or the tiled
//                        kernel of estep_tiled.hip for the common shapes);
//   k_reduce             fixed-order FP64 sum of each dataset's chunk partials;
//   k_mstep              conjugate updates, lower bound, convergence test and
//                        the next E-step's coefficients (update.hip).
#include <math.h>

#include "cavi_impl.h"

namespace cavi {

namespace {

constexpr int kMaxItems = kMaxKG / kBlock;  // (k, g) items per thread

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

// SplitMix64 (Steele, Lea and Flood 2014) and floor(u53 * n / 2^53).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long &s)
{
    unsigned long long z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ unsigned long long scaled_draw(unsigned long long &s, unsigned long long n)
{
    const unsigned long long u = splitmix64(s) >> 11;
    const unsigned long long hi = __umul64hi(u, n), lo = u * n;
    return (hi << 11) | (lo >> 53);
}

// dataset owning a global row (binary search over the datasets' first rows)
__device__ __forceinline__ int dataset_of_row(const Ds *ds, int B, int64_t row)
{
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ds[mid].row0 <= row) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Generic E-step + statistics.  Grid-stride over global chunks; each chunk is
// staged through LDS in tiles of tile_rows rows (row stride G+1 floats).  One
// thread owns one row for the E-step; for the statistics one thread owns
// (k, g) items and walks the tile's rows, skipping rows whose responsibility
// is exactly 0.  init_mode: responsibilities are the hard nearest-seed
// assignment (ties to the lowest seed) instead.
template <int KT>
__global__ __launch_bounds__(kBlock) void k_estep_stats(Shape s, Bufs bf, int init_mode)
{
    extern __shared__ float smem[];
    __shared__ double red[kBlock];
    const int G = s.G;
    const int TR = s.tile_rows, XS = G + 1, RS = KT + 1;
    float *xs = smem;
    float *rs = smem + TR * XS;
    const int tid = threadIdx.x;

    const int nact = n_active_chunks(s, bf);
    for (int slot = blockIdx.x; slot < nact; slot += gridDim.x) {
        const int chunk = active_chunk(s, bf, slot);
        const int bi = bf.chunk_ds[chunk];
        const Ds d = bf.ds[bi];
        if (!init_mode && sweep_skipped(bf.ctl + bi)) continue;
        const int K = d.K, KG = K * G;
        const int nit = (KG + kBlock - 1) / kBlock;
        const size_t kb = (size_t)bi * s.Kmax;
        const float *cc = bf.cc + kb;
        const float2 *hq = (const float2 *)bf.hq + kb * G;
        const float *mf = bf.mf + kb * G;
        float mfv[kMaxItems];
#pragma unroll
        for (int it = 0; it < kMaxItems; ++it) {
            const int p = tid + it * kBlock;
            mfv[it] = (it < nit && p < KG) ? mf[p] : 0.f;
        }
        double a1[kMaxItems], a2[kMaxItems];
#pragma unroll
        for (int it = 0; it < kMaxItems; ++it) a1[it] = a2[it] = 0.0;
        double t0 = 0.0, hh = 0.0;
        const int64_t r0 = d.row0 + (int64_t)(chunk - d.chunk0) * kChunkRows;
        const int64_t r1 = d.row0 + min((int64_t)d.N, (int64_t)(chunk - d.chunk0 + 1) * kChunkRows);
        for (int64_t t = r0; t < r1; t += TR) {
            const int nr = (int)min((int64_t)TR, r1 - t);
            const float *src = bf.x + t * G;
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
                        const uint8_t nb = bf.nearest[t + tid];
                        const int best = nb == kNearestLocked ? 0 : nb;
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
                    const double c = (double)mfv[it];
                    // FP64 sums with exact products (d = x - c formed in FP64), as in the tiled kernel
                    double s1 = 0.0, s2 = 0.0;
                    for (int j = 0; j < nr; ++j) {
                        const float rr = rs[j * RS + k];
                        if (rr != 0.f) {
                            const double dd = (double)xs[j * XS + g] - c;
                            const double w = (double)rr * dd;
                            s1 += w;
                            s2 = fma(w, dd, s2);
                        }
                    }
                    a1[it] += s1;
                    a2[it] += s2;
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
        double *out = bf.partials + (size_t)chunk * s.Smax;
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

// ---------------------------------------------------------------------------------------------
__global__ void k_ctl_begin(int B, Ctl *ctl, int max_call, int stop_on_conv, double tol, int reset)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    Ctl *c = ctl + b;
    c->max_call = max_call;
    c->stop_on_conv = stop_on_conv;
    c->tol = tol;
    c->call_sweeps = 0;
    c->converged = 0;
    c->numeric = 0;
    if (reset) {
        c->sweeps = 0;
        c->elbo = 0.0;
        c->elbo_prev = 0.0;
    }
}

// number of datasets that would still sweep
__global__ void k_count_active(int B, const Ctl *ctl, int32_t *count)
{
    __shared__ int red[kBlock];
    int n = 0;
    for (int b = threadIdx.x; b < B; b += kBlock) n += sweep_skipped(ctl + b) ? 0 : 1;
    red[threadIdx.x] = n;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = red[0];
}

__global__ void k_list_all(Shape s, Bufs bf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        bf.act_n[0] = s.B;
        bf.act_n[1] = s.nchunk;
    }
    if (i < s.B) bf.act_ds[i] = i;
    if (i < s.nchunk) bf.act_chunk[i] = i;
}

// The datasets that will sweep again and their chunks, in ascending order (one workgroup).
// (1) Every dataset's skip test and chunk range are read with independent, coalesced loads
// (thread t takes datasets t, t + 1024, ...) into LDS; (2) each thread takes a contiguous range
// of up to four datasets from LDS, and exclusive scans of their counts (within each wave by lane
// shuffles, then over the 16 wave totals) give the offsets; (3) each thread leaves (list offset,
// first chunk, chunks) of its datasets in LDS by their place in the list, then each wave writes
// whole datasets' chunk ranges (consecutive lanes, consecutive entries).
constexpr int kCompactMaxB = 4096;  // datasets whose entries fit the workgroup's LDS
constexpr int kCompactPer = kCompactMaxB / 1024;

// inclusive scan of v over the 64 lanes of a wave
__device__ __forceinline__ int wave_incl_scan(int v, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

__global__ __launch_bounds__(1024) void k_compact(Shape s, Bufs bf)
{
    __shared__ int l_off[kCompactMaxB], l_c0[kCompactMaxB], l_nc[kCompactMaxB];
    __shared__ int wd[16], wc[16], total;
    if (s.B > kCompactMaxB) return;  // (not launched for such batches: their lists stay whole)
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    // (1) by dataset index: first chunk, and chunks or -1 when the dataset will not sweep
    {
        bool act[kCompactPer];
        Ds d[kCompactPer];
#pragma unroll
        for (int i = 0; i < kCompactPer; ++i) {
            const int b = t + 1024 * i;
            act[i] = false;
            if (b < s.B) {
                act[i] = !sweep_skipped(bf.ctl + b);
                d[i] = bf.ds[b];
            }
        }
#pragma unroll
        for (int i = 0; i < kCompactPer; ++i) {
            const int b = t + 1024 * i;
            if (b < s.B) {
                l_c0[b] = d[i].chunk0;
                l_nc[b] = act[i] ? d[i].nchunk : -1;
            }
        }
    }
    __syncthreads();
    // (2) this thread's contiguous range of datasets
    const int per = (s.B + 1023) / 1024;
    const int b0 = min(s.B, t * per), b1 = min(s.B, b0 + per);
    int c0[kCompactPer], nc[kCompactPer];
    int nd = 0, ncs = 0;
#pragma unroll
    for (int i = 0; i < kCompactPer; ++i) {
        const int b = b0 + i;
        c0[i] = 0;
        nc[i] = -1;
        if (b < b1) {
            c0[i] = l_c0[b];
            nc[i] = l_nc[b];
        }
        if (nc[i] >= 0) {
            ++nd;
            ncs += nc[i];
        }
    }
    const int id = wave_incl_scan(nd, lane), ic = wave_incl_scan(ncs, lane);
    if (lane == 63) {
        wd[wv] = id;
        wc[wv] = ic;
    }
    __syncthreads();  // also ends every read of step (1)'s entries
    if (t < 64) {
        const int vd = lane < 16 ? wd[lane] : 0, vc = lane < 16 ? wc[lane] : 0;
        const int sd = wave_incl_scan(vd, lane), sc = wave_incl_scan(vc, lane);
        if (lane < 16) {
            wd[lane] = sd - vd;  // exclusive offsets of the waves
            wc[lane] = sc - vc;
        }
        if (lane == 15) {
            total = sd;
            bf.act_n[0] = sd;
            bf.act_n[1] = sc;
        }
    }
    __syncthreads();
    int od = wd[wv] + id - nd, oc = wc[wv] + ic - ncs;
#pragma unroll
    for (int i = 0; i < kCompactPer; ++i)
        if (nc[i] >= 0) {
            bf.act_ds[od] = b0 + i;
            l_off[od] = oc;
            l_c0[od] = c0[i];
            l_nc[od] = nc[i];
            ++od;
            oc += nc[i];
        }
    __syncthreads();
    for (int i = wv; i < total; i += 16) {
        const int o = l_off[i], c = l_c0[i], n = l_nc[i];
        for (int k = lane; k < n; k += 64) bf.act_chunk[o + k] = c + k;
    }
}

// ---------------------------------------------------------------------------------------------
// Prior centre m0 = per-gene mean of each dataset: per-chunk FP64 column
// sums, then a fixed-order sum over the dataset's chunks.
__global__ __launch_bounds__(kBlock) void k_colpart(Shape s, Bufs bf)
{
    const int chunk = blockIdx.x, G = s.G;
    const Ds d = bf.ds[bf.chunk_ds[chunk]];
    const int64_t r0 = d.row0 + (int64_t)(chunk - d.chunk0) * kChunkRows;
    const int64_t r1 = d.row0 + min((int64_t)d.N, (int64_t)(chunk - d.chunk0 + 1) * kChunkRows);
    for (int g = threadIdx.x; g < G; g += kBlock) {
        double acc = 0.0;
        for (int64_t r = r0; r < r1; ++r) acc += (double)bf.x[r * G + g];
        bf.colpart[(size_t)chunk * G + g] = acc;
    }
}

// ---------------------------------------------------------------------------------------------
// Passes that read every row of a chunk once (prior centre, k-means++ distances), for G a
// multiple of 4 up to 128: each wave copies RW consecutive rows (contiguous in memory) with
// 16-byte coalesced loads into an LDS slab of its own, of row stride G + 1 (odd, so that a lane
// per row walking its genes and a lane per gene walking the rows both read without bank
// conflicts).  The arithmetic and its order are those of the generic kernels.
template <int G>
struct Slab {
    static constexpr int RW = G <= 64 ? 64 : 32;  // rows per wave slab
    static constexpr int XS = G + 1;              // LDS row stride
    static constexpr int C4 = G / 4;              // 16-byte pieces per row
    static constexpr int PER = (RW * C4 + 63) / 64;
    static_assert(G % 4 == 0 && G <= 128, "staged passes: G a multiple of 4, at most 128");
};

// this wave's LDS operations complete (and none moved across by the compiler)
__device__ __forceinline__ void wave_lds_fence()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

template <int G>
__device__ __forceinline__ void stage_slab(float *xw, const float *src, int nr, int lane)
{
    using S = Slab<G>;
    const float4 *s4 = (const float4 *)src;
    const int n4 = nr * S::C4;
    float4 v[S::PER];
#pragma unroll
    for (int i = 0; i < S::PER; ++i) {
        const int q = lane + 64 * i;
        if (q < n4) v[i] = s4[q];
    }
#pragma unroll
    for (int i = 0; i < S::PER; ++i) {
        const int q = lane + 64 * i;
        if (q < n4) {
            const int r = q / S::C4, c = 4 * (q - r * S::C4);
            float *p = xw + r * S::XS + c;
            p[0] = v[i].x;
            p[1] = v[i].y;
            p[2] = v[i].z;
            p[3] = v[i].w;
        }
    }
    wave_lds_fence();
}

// k_colpart with one wave per chunk (four chunks per workgroup): lane g sums gene g (and
// g + 64) over the chunk's rows in row order
template <int G>
__global__ __launch_bounds__(kBlock) void k_colpart_t(Shape s, Bufs bf)
{
    using S = Slab<G>;
    constexpr int GL = (G + 63) / 64;  // genes per lane
    __shared__ float xs[4][S::RW * S::XS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int chunk = blockIdx.x * 4 + w;
    if (chunk >= s.nchunk) return;  // per wave; no workgroup barrier follows
    const Ds d = bf.ds[bf.chunk_ds[chunk]];
    const int64_t cr = (int64_t)(chunk - d.chunk0) * kChunkRows;
    const int nrc = (int)min((int64_t)kChunkRows, (int64_t)d.N - cr);
    float *xw = xs[w];
    double acc[GL];
#pragma unroll
    for (int i = 0; i < GL; ++i) acc[i] = 0.0;
    for (int r0 = 0; r0 < nrc; r0 += S::RW) {
        const int nr = min(S::RW, nrc - r0);
        stage_slab<G>(xw, bf.x + (d.row0 + cr + r0) * G, nr, lane);
        for (int r = 0; r < nr; ++r)
#pragma unroll
            for (int i = 0; i < GL; ++i) {
                const int g = lane + 64 * i;
                if (g < G) acc[i] += (double)xw[r * S::XS + g];
            }
        wave_lds_fence();  // the slab is read before the next one overwrites it
    }
#pragma unroll
    for (int i = 0; i < GL; ++i) {
        const int g = lane + 64 * i;
        if (g < G) bf.colpart[(size_t)chunk * G + g] = acc[i];
    }
}

__global__ __launch_bounds__(kBlock) void k_colmean(Shape s, Bufs bf)
{
    const int bi = blockIdx.x, G = s.G;
    const Ds d = bf.ds[bi];
    for (int g = threadIdx.x; g < G; g += kBlock) {
        double acc = 0.0;
        for (int c = d.chunk0; c < d.chunk0 + d.nchunk; ++c) acc += bf.colpart[(size_t)c * G + g];
        bf.m0[(size_t)bi * G + g] = acc / (double)d.N;
    }
}

// ---------------------------------------------------------------------------------------------
// k-means++ seeds (D^2 sampling) of every dataset of a batch, on the device, with many
// workgroups per dataset: one pass over all rows per seed.  Definition (shared with the
// oracle): the SplitMix64 state of dataset b draws the first seed row floor(u N); each later
// seed is the smallest row whose cumulative integer weight floor(minD2 2^e) exceeds
// floor(u W), W the sum of the weights and e = 62 - E - ceil(log2 N) for the largest minD2 =
// f 2^E (f in [1/2, 1)); if every minD2 is 0 the row is floor(u N) again.  minD2 is the FP64
// squared distance to the nearest seed so far, genes added in order.
//
// Per-dataset state, in the totals array (free during initialisation):
//   [0] SplitMix64 state, [1] chosen row, [2] e (or kNoWeights when every minD2 is 0).
// Per-chunk maxima and weight sums: blockmax / blocksum, indexed by the global chunk.
namespace {
constexpr long long kNoWeights = -1000000;

__device__ __forceinline__ unsigned long long *pp_state(const Shape &s, const Bufs &bf, int bi)
{
    return (unsigned long long *)(bf.totals + (size_t)bi * s.Smax);
}

__device__ __forceinline__ int ceil_log2(int64_t n)
{
    int c = 0;
    while (((int64_t)1 << c) < n) ++c;
    return c;
}

// inclusive prefix sum over the 64 lanes of a wave (exact: integers)
__device__ __forceinline__ unsigned long long wave_scan(unsigned long long v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}
}  // namespace

__global__ void k_pp_begin(Shape s, Bufs bf, unsigned long long seed)
{
    const int bi = blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= s.B) return;
    unsigned long long *st = pp_state(s, bf, bi);
    unsigned long long rng = seed + (unsigned long long)bi;
    st[1] = scaled_draw(rng, (unsigned long long)bf.ds[bi].N);
    st[0] = rng;
}

// The hard assignment's nearest seed, kept during the distance passes: the first minimum of the
// sequential scan over the seeds (seed 0 taken first, a later seed only when strictly nearer
// than every earlier one, so a NaN distance never replaces; a NaN distance to seed 0 keeps seed 0
// whatever follows).  The distances are the passes' own FP64 values, genes added in order, so
// this is the nearest seed by that definition.  `old` is the smallest distance of the earlier
// seeds, as minD2 holds it (minD2 ignores NaN distances, as the scan does after seed 0).
__device__ __forceinline__ void update_nearest(uint8_t *p, int j, double acc, double old)
{
    if (j == 0) {
        *p = acc != acc ? kNearestLocked : 0;
    } else {
        const uint8_t o = *p;
        if (o != kNearestLocked && acc < old) *p = (uint8_t)j;
    }
}

// one workgroup per chunk: minD2 against seed j (rows staged through LDS 32 genes at a time),
// the chunk maximum, and the copy of the seed row into the seed table
__global__ __launch_bounds__(kBlock) void k_pp_d2(Shape s, Bufs bf, int j)
{
    constexpr int kSlab = 32;
    __shared__ float xs[kBlock][kSlab + 1];
    __shared__ float sd[kSlab];
    __shared__ double red[kBlock];
    const int chunk = blockIdx.x, tid = threadIdx.x, G = s.G;
    const int bi = bf.chunk_ds[chunk];
    const Ds d = bf.ds[bi];
    if (j >= d.K) return;
    const int64_t row = (int64_t)pp_state(s, bf, bi)[1];
    const float *seed = bf.x + (d.row0 + row) * G;
    if (chunk == d.chunk0)
        for (int g = tid; g < G; g += kBlock) bf.seeds[((size_t)bi * s.Kmax + j) * G + g] = seed[g];
    const int64_t c0 = (int64_t)(chunk - d.chunk0) * kChunkRows;
    const int nrc = (int)min((int64_t)kChunkRows, (int64_t)d.N - c0);
    double mx = 0.0;
    for (int r0 = 0; r0 < nrc; r0 += kBlock) {
        const int nr = min(kBlock, nrc - r0);
        const float *xb = bf.x + (d.row0 + c0 + r0) * G;
        double acc = 0.0;
        for (int g0 = 0; g0 < G; g0 += kSlab) {
            const int w = min(kSlab, G - g0);
            for (int e = tid; e < kBlock * kSlab; e += kBlock) {
                const int r = e / kSlab, c = e - r * kSlab;
                if (r < nr && c < w) xs[r][c] = xb[(int64_t)r * G + g0 + c];
            }
            if (tid < w) sd[tid] = seed[g0 + tid];
            __syncthreads();
            if (tid < nr) {
#pragma clang fp contract(off)
                for (int c = 0; c < w; ++c) {
                    const double dd = (double)xs[tid][c] - (double)sd[c];
                    acc = acc + dd * dd;
                }
            }
            __syncthreads();
        }
        if (tid < nr) {
            double *m = bf.mind2 + d.row0 + c0 + r0 + tid;
            const double old = j == 0 ? acc : *m;
            const double v = j == 0 ? acc : fmin(old, acc);
            *m = v;
            mx = fmax(mx, v);
            update_nearest(bf.nearest + d.row0 + c0 + r0 + tid, j, acc, old);
        }
    }
    red[tid] = mx;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (tid < off) red[tid] = fmax(red[tid], red[tid + off]);
        __syncthreads();
    }
    if (tid == 0) bf.blockmax[chunk] = red[0];
}

// k_pp_d2 for G a multiple of 4 up to 128: each wave stages its own slabs of the chunk, a lane
// per row
template <int G>
__global__ __launch_bounds__(kBlock) void k_pp_d2_t(Shape s, Bufs bf, int j)
{
    using S = Slab<G>;
    __shared__ float xs[4][S::RW * S::XS];
    __shared__ double sd[G];
    __shared__ double red[4];
    const int chunk = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int bi = bf.chunk_ds[chunk];
    const Ds d = bf.ds[bi];
    if (j >= d.K) return;
    const int64_t row = (int64_t)pp_state(s, bf, bi)[1];
    const float *seed = bf.x + (d.row0 + row) * G;
    if (chunk == d.chunk0)
        for (int g = tid; g < G; g += kBlock) bf.seeds[((size_t)bi * s.Kmax + j) * G + g] = seed[g];
    for (int g = tid; g < G; g += kBlock) sd[g] = (double)seed[g];
    __syncthreads();
    const int64_t cr = (int64_t)(chunk - d.chunk0) * kChunkRows;
    const int nrc = (int)min((int64_t)kChunkRows, (int64_t)d.N - cr);
    float *xw = xs[w];
    double mx = 0.0;
    for (int r0 = w * S::RW; r0 < nrc; r0 += 4 * S::RW) {
        const int nr = min(S::RW, nrc - r0);
        stage_slab<G>(xw, bf.x + (d.row0 + cr + r0) * G, nr, lane);
        if (lane < nr) {
#pragma clang fp contract(off)
            const float *xr = xw + lane * S::XS;
            double acc = 0.0;
            for (int g = 0; g < G; ++g) {
                const double dd = (double)xr[g] - sd[g];
                acc = acc + dd * dd;
            }
            double *m = bf.mind2 + d.row0 + cr + r0 + lane;
            const double old = j == 0 ? acc : *m;
            const double v = j == 0 ? acc : fmin(old, acc);
            *m = v;
            mx = fmax(mx, v);
            update_nearest(bf.nearest + d.row0 + cr + r0 + lane, j, acc, old);
        }
        wave_lds_fence();  // the slab is read before the next one overwrites it
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) red[w] = mx;
    __syncthreads();
    if (tid == 0) bf.blockmax[chunk] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// one wave per dataset: e from the largest minD2 of its chunks
__global__ __launch_bounds__(64) void k_pp_exp(Shape s, Bufs bf, int j)
{
    const int bi = blockIdx.x, lane = threadIdx.x;
    const Ds d = bf.ds[bi];
    if (j >= d.K) return;
    double mx = 0.0;
    for (int c = lane; c < d.nchunk; c += 64) mx = fmax(mx, bf.blockmax[d.chunk0 + c]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) {
        long long e = kNoWeights;
        if (mx > 0.0) {
            int E;
            frexp(mx, &E);
            e = 62 - E - ceil_log2(d.N);
        }
        pp_state(s, bf, bi)[2] = (unsigned long long)e;
    }
}

// one workgroup per chunk: sum of the integer weights floor(minD2 2^e)
__global__ __launch_bounds__(kBlock) void k_pp_wsum(Shape s, Bufs bf, int j)
{
    __shared__ unsigned long long red[kBlock];
    const int chunk = blockIdx.x, tid = threadIdx.x;
    const int bi = bf.chunk_ds[chunk];
    const Ds d = bf.ds[bi];
    if (j >= d.K) return;
    const long long e = (long long)pp_state(s, bf, bi)[2];
    if (e == kNoWeights) return;
    const int64_t c0 = (int64_t)(chunk - d.chunk0) * kChunkRows;
    const int nrc = (int)min((int64_t)kChunkRows, (int64_t)d.N - c0);
    const double *m = bf.mind2 + d.row0 + c0;
    unsigned long long w = 0;
    for (int r = tid; r < nrc; r += kBlock) w += (unsigned long long)floor(ldexp(m[r], (int)e));
    red[tid] = w;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    if (tid == 0) bf.blocksum[chunk] = red[0];
}

// one wave per dataset: the draw for seed j; the chunk holding it, then the row
__global__ __launch_bounds__(64) void k_pp_draw(Shape s, Bufs bf, int j)
{
    const int bi = blockIdx.x, lane = threadIdx.x;
    const Ds d = bf.ds[bi];
    if (j >= d.K) return;
    unsigned long long *st = pp_state(s, bf, bi);
    unsigned long long rng = st[0];
    const long long e = (long long)st[2];
    if (e == kNoWeights) {
        const unsigned long long r = scaled_draw(rng, (unsigned long long)d.N);
        if (lane == 0) {
            st[1] = r;
            st[0] = rng;
        }
        return;
    }
    unsigned long long W = 0;
    for (int c = lane; c < d.nchunk; c += 64) W += bf.blocksum[d.chunk0 + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) W += __shfl_xor(W, off, 64);
    const unsigned long long t = scaled_draw(rng, W);  // every lane: same state, same draw
    // chunk: the first whose cumulative sum exceeds t
    unsigned long long base = 0;
    int ch = d.nchunk - 1;
    for (int c0 = 0; c0 < d.nchunk; c0 += 64) {
        const int c = c0 + lane;
        const unsigned long long v = c < d.nchunk ? bf.blocksum[d.chunk0 + c] : 0ull;
        const unsigned long long cum = base + wave_scan(v);
        const unsigned long long hit = __ballot(c < d.nchunk && cum > t);
        if (hit) {
            const int l = __builtin_ctzll(hit);
            ch = c0 + l;
            base = __shfl(cum, l, 64) - __shfl(v, l, 64);
            break;
        }
        base = __shfl(cum, 63, 64);
    }
    // row within the chunk
    const int64_t r0 = (int64_t)ch * kChunkRows;
    const int nrc = (int)min((int64_t)kChunkRows, (int64_t)d.N - r0);
    const double *m = bf.mind2 + d.row0 + r0;
    int64_t row = r0 + nrc - 1;
    for (int q0 = 0; q0 < nrc; q0 += 64) {
        const int q = q0 + lane;
        const unsigned long long v = q < nrc ? (unsigned long long)floor(ldexp(m[q], (int)e)) : 0ull;
        const unsigned long long cum = base + wave_scan(v);
        const unsigned long long hit = __ballot(q < nrc && cum > t);
        if (hit) {
            row = r0 + q0 + __builtin_ctzll(hit);
            break;
        }
        base = __shfl(cum, 63, 64);
    }
    if (lane == 0) {
        st[1] = (unsigned long long)row;
        st[0] = rng;
    }
}

// ---------------------------------------------------------------------------------------------
// Responsibilities of the current coefficients, one thread per row; r is
// Ntot x Kmax (row-major), entries k >= K of a dataset are left untouched.
template <int KT>
__global__ __launch_bounds__(kBlock) void k_resp(Shape s, Bufs bf, float *__restrict__ r)
{
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= s.Ntot) return;
    const int bi = dataset_of_row(bf.ds, s.B, n);
    const int K = bf.ds[bi].K;
    const size_t kb = (size_t)bi * s.Kmax;
    float l[KT];
    row_loglik<KT>(bf.x + n * s.G, s.G, K, (const float2 *)bf.hq + kb * s.G, bf.cc + kb, l);
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
            r[n * s.Kmax + k] = dl > -kLogRCut ? __expf(dl) : 0.f;
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
    const size_t B = s.B, K = (size_t)s.B * s.Kmax, KG = K * s.G, G = s.G;
    const size_t nblk = s.nchunk;  // per-chunk maxima and weight sums (initialisation)
    size_t n = 0;
    n += al(B * sizeof(Ds)) + al((size_t)s.nchunk * 4);
    n += al(K * 8);                    // alpha
    n += 8 * al(KG * 8);               // m beta a b, nm nbeta na nb
    n += al(B * G * 8);                // m0
    n += al(K * 4) + al(2 * KG * 4) + 2 * al(KG * 4);  // cc, hq, mf, seeds
    n += al((size_t)s.nchunk * s.Smax * 8);
    n += al(B * red_split_max(s.Nmax) * s.Smax * 8);  // totals
    n += al(B * s.hist_cap * 8);
    n += al(B * sizeof(Ctl)) + al(4);
    n += al((size_t)s.Ntot * 8) + al((size_t)s.Ntot);  // mind2, nearest
    n += 2 * al(nblk * 8);
    n += al((size_t)s.nchunk * G * 8);
    n += al(2 * 4) + al(B * 4) + al((size_t)s.nchunk * 4);  // work lists
    return n;
}

void carve(const Shape &s, void *ws, Bufs &b)
{
    const size_t B = s.B, K = (size_t)s.B * s.Kmax, KG = K * s.G, G = s.G;
    const size_t nblk = s.nchunk;  // per-chunk maxima and weight sums (initialisation)
    char *p = (char *)ws;
    auto take = [&](size_t bytes) {
        void *r = p;
        p += al(bytes);
        return r;
    };
    b.ds = (const Ds *)take(B * sizeof(Ds));
    b.chunk_ds = (const int32_t *)take((size_t)s.nchunk * 4);
    b.alpha = (double *)take(K * 8);
    b.m = (double *)take(KG * 8);
    b.beta = (double *)take(KG * 8);
    b.a = (double *)take(KG * 8);
    b.b = (double *)take(KG * 8);
    b.nm = (double *)take(KG * 8);
    b.nbeta = (double *)take(KG * 8);
    b.na = (double *)take(KG * 8);
    b.nb = (double *)take(KG * 8);
    b.m0 = (double *)take(B * G * 8);
    b.cc = (float *)take(K * 4);
    b.hq = (float *)take(2 * KG * 4);
    b.mf = (float *)take(KG * 4);
    b.seeds = (float *)take(KG * 4);
    b.partials = (double *)take((size_t)s.nchunk * s.Smax * 8);
    b.totals = (double *)take(B * red_split_max(s.Nmax) * s.Smax * 8);
    b.hist = (double *)take(B * s.hist_cap * 8);
    b.ctl = (Ctl *)take(B * sizeof(Ctl));
    b.count = (int32_t *)take(4);
    b.mind2 = (double *)take((size_t)s.Ntot * 8);
    b.nearest = (uint8_t *)take((size_t)s.Ntot);
    b.blockmax = (double *)take(nblk * 8);
    b.blocksum = (unsigned long long *)take(nblk * 8);
    b.colpart = (double *)take((size_t)s.nchunk * G * 8);
    b.act_n = (int32_t *)take(2 * 4);
    b.act_ds = (int32_t *)take(B * 4);
    b.act_chunk = (int32_t *)take((size_t)s.nchunk * 4);
}

int g_lds_limit = 0;

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
    // tile size is chosen against the limit that the device reports.
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

// Plain streaming read of n floats (16-byte loads, grid-stride, four loads in flight per lane);
// each workgroup writes the sum of what it read so that the loads are kept.
__global__ __launch_bounds__(kBlock) void k_read_probe(const float4 *__restrict__ x, int64_t n4,
                                                       const float *__restrict__ tail, int ntail, float *out)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    float acc = 0.f;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 a = x[i], b = x[i + stride], c = x[i + 2 * stride], d = x[i + 3 * stride];
        acc += ((a.x + b.x) + (c.x + d.x)) + ((a.y + b.y) + (c.y + d.y)) + ((a.z + b.z) + (c.z + d.z)) +
               ((a.w + b.w) + (c.w + d.w));
    }
    for (; i < n4; i += stride) {
        const float4 a = x[i];
        acc += (a.x + a.y) + (a.z + a.w);
    }
    if (blockIdx.x == 0 && threadIdx.x < ntail) acc += tail[threadIdx.x];
    __shared__ float red[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

hipError_t launch_read_probe(const float *x, int64_t n, float *out, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_read_probe, dim3(grid), dim3(kBlock), 0, st, (const float4 *)x, n / 4, x + (n / 4) * 4,
                       (int)(n % 4), out);
    return hipGetLastError();
}

template <int KT>
static hipError_t launch_estep_t(const Shape &s, const Bufs &b, int init_mode, hipStream_t st)
{
    const size_t lds = (size_t)s.tile_rows * (s.G + 1 + KT + 1) * sizeof(float);
    hipLaunchKernelGGL(k_estep_stats<KT>, dim3(s.egrid), dim3(kBlock), lds, st, s, b, init_mode);
    return hipGetLastError();
}

hipError_t launch_estep_stats(const Shape &s, const Bufs &b, int init_mode, hipStream_t st)
{
    if (tiled_supported(s.Kmax, s.G)) return launch_estep_tiled(s, b, init_mode, st);
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
    const dim3 g4((s.nchunk + 3) / 4);
    switch (s.G) {
    case 16: hipLaunchKernelGGL(k_colpart_t<16>, g4, dim3(kBlock), 0, st, s, b); break;
    case 32: hipLaunchKernelGGL(k_colpart_t<32>, g4, dim3(kBlock), 0, st, s, b); break;
    case 48: hipLaunchKernelGGL(k_colpart_t<48>, g4, dim3(kBlock), 0, st, s, b); break;
    case 64: hipLaunchKernelGGL(k_colpart_t<64>, g4, dim3(kBlock), 0, st, s, b); break;
    case 96: hipLaunchKernelGGL(k_colpart_t<96>, g4, dim3(kBlock), 0, st, s, b); break;
    case 128: hipLaunchKernelGGL(k_colpart_t<128>, g4, dim3(kBlock), 0, st, s, b); break;
    default: hipLaunchKernelGGL(k_colpart, dim3(s.nchunk), dim3(kBlock), 0, st, s, b); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colmean, dim3(s.B), dim3(kBlock), 0, st, s, b);
    return hipGetLastError();
}

hipError_t launch_kmeanspp(const Shape &s, const Bufs &b, unsigned long long seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_pp_begin, dim3((s.B + 255) / 256), dim3(256), 0, st, s, b, seed);
    for (int j = 0; j < s.Kmax; ++j) {
        if (j > 0) {
            hipLaunchKernelGGL(k_pp_exp, dim3(s.B), dim3(64), 0, st, s, b, j);
            hipLaunchKernelGGL(k_pp_wsum, dim3(s.nchunk), dim3(kBlock), 0, st, s, b, j);
            hipLaunchKernelGGL(k_pp_draw, dim3(s.B), dim3(64), 0, st, s, b, j);
        }
        const dim3 gc(s.nchunk), bk(kBlock);
        switch (s.G) {
        case 16: hipLaunchKernelGGL(k_pp_d2_t<16>, gc, bk, 0, st, s, b, j); break;
        case 32: hipLaunchKernelGGL(k_pp_d2_t<32>, gc, bk, 0, st, s, b, j); break;
        case 48: hipLaunchKernelGGL(k_pp_d2_t<48>, gc, bk, 0, st, s, b, j); break;
        case 64: hipLaunchKernelGGL(k_pp_d2_t<64>, gc, bk, 0, st, s, b, j); break;
        case 96: hipLaunchKernelGGL(k_pp_d2_t<96>, gc, bk, 0, st, s, b, j); break;
        case 128: hipLaunchKernelGGL(k_pp_d2_t<128>, gc, bk, 0, st, s, b, j); break;
        default: hipLaunchKernelGGL(k_pp_d2, gc, bk, 0, st, s, b, j); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_resp(const Shape &s, const Bufs &b, float *r, hipStream_t st)
{
    const dim3 grid((unsigned)((s.Ntot + kBlock - 1) / kBlock));
    switch (s.kt) {
    case 4: hipLaunchKernelGGL(k_resp<4>, grid, dim3(kBlock), 0, st, s, b, r); break;
    case 8: hipLaunchKernelGGL(k_resp<8>, grid, dim3(kBlock), 0, st, s, b, r); break;
    case 16: hipLaunchKernelGGL(k_resp<16>, grid, dim3(kBlock), 0, st, s, b, r); break;
    case 32: hipLaunchKernelGGL(k_resp<32>, grid, dim3(kBlock), 0, st, s, b, r); break;
    default: hipLaunchKernelGGL(k_resp<64>, grid, dim3(kBlock), 0, st, s, b, r); break;
    }
    return hipGetLastError();
}

hipError_t launch_ctl_begin(const Shape &s, const Bufs &b, int max_call, int stop_on_conv, double tol, int reset,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_ctl_begin, dim3((s.B + 255) / 256), dim3(256), 0, st, s.B, b.ctl, max_call, stop_on_conv,
                       tol, reset);
    return hipGetLastError();
}

hipError_t launch_count_active(const Shape &s, const Bufs &b, hipStream_t st)
{
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(kBlock), 0, st, s.B, b.ctl, b.count);
    return hipGetLastError();
}

hipError_t launch_list_all(const Shape &s, const Bufs &b, hipStream_t st)
{
    const int n = s.nchunk > s.B ? s.nchunk : s.B;
    hipLaunchKernelGGL(k_list_all, dim3((n + 255) / 256), dim3(256), 0, st, s, b);
    return hipGetLastError();
}

hipError_t launch_compact(const Shape &s, const Bufs &b, hipStream_t st)
{
    if (s.B > kCompactMaxB) return hipSuccess;  // such a batch sweeps over its whole lists
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, st, s, b);
    return hipGetLastError();
}

}  // namespace cavi
