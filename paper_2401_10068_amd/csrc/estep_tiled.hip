// Tiled E-step + statistics kernel for the common shapes (G a multiple of 4
// up to 128, K up to 16): the same arithmetic as k_estep_stats, organised for
// gfx950.
//
// Per 2048-row chunk (the unit of the deterministic reduction), 128-row tiles
// are staged in LDS (row stride G+4 floats; the next tile is prefetched into
// registers while the current one is processed).  Per tile:
//   1. E-step.  Wave w owns subpopulations k = w, w+4, ...; each lane owns
//      two rows.  The coefficients of k are wave-uniform, so they arrive by
//      scalar loads: l_nk = c_k - sum_g (h_kg x_ng + q_kg)^2.
//   2. Log-sum-exp.  One thread per row: L_n, r_nk = exp(l_nk - L_n) (zero
//      below exp(-87)), the entropy term, and a bitmask of the nonzero r_nk.
//   3. Statistics.  Wave w walks rows 32w..32w+31, lanes over genes; for each
//      subpopulation in the row's mask (a uniform scalar branch):
//      T0 += r,  T1 += r d,  T2 += r d^2  with d = x - m_kg (FP32 centre).
// Each wave sums its 512 rows of a chunk in FP32 (the sums are taken around
// the previous mean, so they do not cancel); the four wave sums are promoted
// to FP64 and added in wave order; the chunk partial is T0 | T1 | T2 | H.
#include <math.h>

#include "cavi_impl.h"

namespace cavi {

namespace {

constexpr int kT = 128;        // rows per tile
typedef float f4 __attribute__((ext_vector_type(4)));

template <int KT, int G>
struct Cfg {
    static constexpr int XS = G + 4;                     // LDS row stride of the x tile
    static constexpr int LS = (KT == 4) ? 12 : KT + 4;   // LDS row stride of l / r
    static constexpr int KQ = KT / 4;                    // subpopulations per wave (E-step)
    static constexpr int GS = (G + 63) / 64;             // gene slots per lane (statistics)
    static constexpr int LOADS = (kT * G / 4) / kBlock;  // float4 loads per thread per tile
    static constexpr int LDS_BYTES = (kT * XS + kT * LS) * 4 + kT * 4;
    static_assert(G % 4 == 0, "G must be a multiple of 4");
    static_assert((kT * G / 4) % kBlock == 0, "tile must split evenly into float4 loads");
    static_assert((KT + 2 * KT * G) * 8 <= kT * XS * 4, "chunk combine must fit the x tile");
};

template <int G>
__device__ __forceinline__ void load_tile(f4 (&pre)[(kT * G / 4) / kBlock], const float *__restrict__ x,
                                          int64_t row0, int nr, int tid)
{
    constexpr int C4 = G / 4;
#pragma unroll
    for (int j = 0; j < (kT * G / 4) / kBlock; ++j) {
        const int i = tid + j * kBlock;
        const int row = i / C4;
        const int col = (i - row * C4) * 4;
        if (row < nr) pre[j] = *(const f4 *)(x + (row0 + row) * G + col);
    }
}

template <int G>
__device__ __forceinline__ void store_tile(const f4 (&pre)[(kT * G / 4) / kBlock], float *xs, int nr, int tid)
{
    constexpr int C4 = G / 4, XS = G + 4;
#pragma unroll
    for (int j = 0; j < (kT * G / 4) / kBlock; ++j) {
        const int i = tid + j * kBlock;
        const int row = i / C4;
        const int col = (i - row * C4) * 4;
        if (row < nr) *(f4 *)(xs + row * XS + col) = pre[j];
    }
}

}  // namespace

template <int KT, int G>
__global__ __launch_bounds__(kBlock, 2) void k_estep_tiled(Shape s, const float *__restrict__ x,
                                                           const float *__restrict__ cc,
                                                           const float *__restrict__ hq,
                                                           const float *__restrict__ mf,
                                                           double *__restrict__ partials,
                                                           const Ctl *__restrict__ ctl)
{
    using C = Cfg<KT, G>;
    constexpr int XS = C::XS, LS = C::LS, KQ = C::KQ, GS = C::GS;
    if (sweep_skipped(ctl)) return;
    extern __shared__ __align__(16) float smem[];
    float *xs = smem;
    float *ls = xs + kT * XS;
    uint32_t *msk = (uint32_t *)(ls + kT * LS);
    __shared__ double red[kBlock];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int K = s.K, KG = K * G;

    float mfv[KT][GS];
#pragma unroll
    for (int k = 0; k < KT; ++k)
#pragma unroll
        for (int sl = 0; sl < GS; ++sl) {
            const int g = lane + 64 * sl;
            mfv[k][sl] = (k < K && g < G) ? mf[k * G + g] : 0.f;
        }

    for (int chunk = blockIdx.x; chunk < s.nchunk; chunk += gridDim.x) {
        const int64_t r0 = (int64_t)chunk * kChunkRows;
        const int nrc = (int)min((int64_t)kChunkRows, s.N - r0);
        const int ntiles = (nrc + kT - 1) / kT;

        float t0[KT], t1[KT][GS], t2[KT][GS];
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            t0[k] = 0.f;
#pragma unroll
            for (int sl = 0; sl < GS; ++sl) t1[k][sl] = t2[k][sl] = 0.f;
        }
        double hacc = 0.0;

        f4 pre[C::LOADS];
        load_tile<G>(pre, x, r0, min(kT, nrc), tid);
        for (int t = 0; t < ntiles; ++t) {
            const int nr = min(kT, nrc - t * kT);
            store_tile<G>(pre, xs, nr, tid);
            __syncthreads();
            if (t + 1 < ntiles) load_tile<G>(pre, x, r0 + (int64_t)(t + 1) * kT, min(kT, nrc - (t + 1) * kT), tid);

            // 1. E-step: sums of squares for rows lane and lane+64, subpopulations w + 4i
            {
                float acc0[KQ], acc1[KQ];
#pragma unroll
                for (int i = 0; i < KQ; ++i) acc0[i] = acc1[i] = 0.f;
                const float *xa = xs + lane * XS;
                const float *xb = xs + (lane + 64) * XS;
#pragma unroll 4
                for (int gb = 0; gb < G; gb += 4) {
                    const f4 va = *(const f4 *)(xa + gb);
                    const f4 vb = *(const f4 *)(xb + gb);
#pragma unroll
                    for (int i = 0; i < KQ; ++i) {
                        const int k = w + 4 * i;
                        if (k < K) {
                            const float *p = hq + 2 * (k * G + gb);
                            const float h0 = p[0], q0 = p[1], h1 = p[2], q1 = p[3];
                            const float h2 = p[4], q2 = p[5], h3 = p[6], q3 = p[7];
                            float u;
                            u = fmaf(va.x, h0, q0); acc0[i] = fmaf(u, u, acc0[i]);
                            u = fmaf(vb.x, h0, q0); acc1[i] = fmaf(u, u, acc1[i]);
                            u = fmaf(va.y, h1, q1); acc0[i] = fmaf(u, u, acc0[i]);
                            u = fmaf(vb.y, h1, q1); acc1[i] = fmaf(u, u, acc1[i]);
                            u = fmaf(va.z, h2, q2); acc0[i] = fmaf(u, u, acc0[i]);
                            u = fmaf(vb.z, h2, q2); acc1[i] = fmaf(u, u, acc1[i]);
                            u = fmaf(va.w, h3, q3); acc0[i] = fmaf(u, u, acc0[i]);
                            u = fmaf(vb.w, h3, q3); acc1[i] = fmaf(u, u, acc1[i]);
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < KQ; ++i) {
                    const int k = w + 4 * i;
                    if (k < K) {
                        ls[lane * LS + k] = acc0[i];
                        ls[(lane + 64) * LS + k] = acc1[i];
                    }
                }
            }
            __syncthreads();

            // 2. log-sum-exp for the wave's own 32 rows (lane jj < 32 owns row 32w + jj):
            //    responsibilities stay in registers, with a bitmask of the nonzero ones.
            const int jbase = 32 * w;
            const int nj = max(0, min(32, nr - jbase));
            float rv[KT];
            uint32_t mk = 0;
#pragma unroll
            for (int k = 0; k < KT; ++k) rv[k] = 0.f;
            if (lane < nj) {
                const float *lr = ls + (jbase + lane) * LS;
                float l[KT];
#pragma unroll
                for (int k = 0; k < KT; ++k) l[k] = (k < K) ? cc[k] - lr[k] : -INFINITY;
                float mx = l[0];
#pragma unroll
                for (int k = 1; k < KT; ++k) mx = fmaxf(mx, l[k]);
                float se = 0.f;
#pragma unroll
                for (int k = 0; k < KT; ++k)
                    if (k < K) se += __expf(l[k] - mx);
                const float L = mx + __logf(se);
                float h = isfinite(L) ? 0.f : __int_as_float(0x7fc00000);
#pragma unroll
                for (int k = 0; k < KT; ++k) {
                    if (k < K) {
                        const float dl = l[k] - L;
                        if (dl > -kLogRCut) {
                            rv[k] = __expf(dl);
                            h -= rv[k] * dl;
                        }
                    }
                    if (rv[k] != 0.f) mk |= 1u << k;
                }
                hacc += (double)h;
            }

            // 3. statistics over the same rows, lanes over genes; the row's mask and
            //    responsibilities are read across lanes into scalar registers.
            if (nj > 0) {
                float xv[GS];
#pragma unroll
                for (int sl = 0; sl < GS; ++sl) {
                    const int g = lane + 64 * sl;
                    xv[sl] = (g < G) ? xs[jbase * XS + g] : 0.f;
                }
                for (int jj = 0; jj < nj; ++jj) {
                    float xn[GS];
                    const int jn = jbase + min(jj + 1, nj - 1);
#pragma unroll
                    for (int sl = 0; sl < GS; ++sl) {
                        const int g = lane + 64 * sl;
                        xn[sl] = (g < G) ? xs[jn * XS + g] : 0.f;
                    }
                    const uint32_t m = (uint32_t)__builtin_amdgcn_readlane((int)mk, jj);
#pragma unroll
                    for (int k = 0; k < KT; ++k) {
                        if (m & (1u << k)) {
                            const float r = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rv[k]), jj));
                            t0[k] += r;
#pragma unroll
                            for (int sl = 0; sl < GS; ++sl) {
                                const float d = xv[sl] - mfv[k][sl];
                                const float wv = r * d;
                                t1[k][sl] += wv;
                                t2[k][sl] = fmaf(wv, d, t2[k][sl]);
                            }
                        }
                    }
#pragma unroll
                    for (int sl = 0; sl < GS; ++sl) xv[sl] = xn[sl];
                }
            }
            __syncthreads();
        }

        // combine the four waves in wave order (FP64, in the LDS of the x tile)
        double *cb = (double *)smem;
        for (int ww = 0; ww < 4; ++ww) {
            if (w == ww) {
#pragma unroll
                for (int k = 0; k < KT; ++k) {
                    if (k < K) {
                        if (lane == 0) cb[k] = (ww == 0) ? (double)t0[k] : cb[k] + (double)t0[k];
#pragma unroll
                        for (int sl = 0; sl < GS; ++sl) {
                            const int g = lane + 64 * sl;
                            if (g < G) {
                                const int i1 = K + k * G + g, i2 = K + KG + k * G + g;
                                cb[i1] = (ww == 0) ? (double)t1[k][sl] : cb[i1] + (double)t1[k][sl];
                                cb[i2] = (ww == 0) ? (double)t2[k][sl] : cb[i2] + (double)t2[k][sl];
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
        red[tid] = hacc;
        __syncthreads();
        for (int off = kBlock / 2; off > 0; off >>= 1) {
            if (tid < off) red[tid] += red[tid + off];
            __syncthreads();
        }
        double *out = partials + (size_t)chunk * s.S;
        for (int i = tid; i < K + 2 * KG; i += kBlock) out[i] = cb[i];
        if (tid == 0) out[K + 2 * KG] = red[0];
        __syncthreads();
    }
}

namespace {

template <int KT, int G>
hipError_t launch_t(const Shape &s, const Bufs &b, hipStream_t st)
{
    constexpr int lds = Cfg<KT, G>::LDS_BYTES;
    hipLaunchKernelGGL((k_estep_tiled<KT, G>), dim3(s.nchunk), dim3(kBlock), lds, st, s, b.x, b.cc, b.hq, b.mf,
                       b.partials, b.ctl);
    return hipGetLastError();
}

template <int KT>
hipError_t launch_g(const Shape &s, const Bufs &b, hipStream_t st)
{
    switch (s.G) {
    case 16: return launch_t<KT, 16>(s, b, st);
    case 32: return launch_t<KT, 32>(s, b, st);
    case 48: return launch_t<KT, 48>(s, b, st);
    case 64: return launch_t<KT, 64>(s, b, st);
    case 96: return launch_t<KT, 96>(s, b, st);
    case 128: return launch_t<KT, 128>(s, b, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool tiled_supported(int K, int G)
{
    const bool g_ok = G == 16 || G == 32 || G == 48 || G == 64 || G == 96 || G == 128;
    if (!g_ok) return false;
    const int kt = choose_kt(K);
    const int gs = (G + 63) / 64;
    if (kt > 16 || kt * gs > 16) return false;
    const int ls = (kt == 4) ? 12 : kt + 4;
    const int bytes = (kT * (G + 4) + kT * ls) * 4 + kT * 4 + kBlock * 8;
    return bytes <= (g_lds_limit > 0 ? g_lds_limit : 65536);
}

hipError_t launch_estep_tiled(const Shape &s, const Bufs &b, hipStream_t st)
{
    switch (s.kt) {
    case 4: return launch_g<4>(s, b, st);
    case 8: return launch_g<8>(s, b, st);
    case 16:
        switch (s.G) {
        case 16: return launch_t<16, 16>(s, b, st);
        case 32: return launch_t<16, 32>(s, b, st);
        case 48: return launch_t<16, 48>(s, b, st);
        case 64: return launch_t<16, 64>(s, b, st);
        default: return hipErrorInvalidValue;
        }
    default: return hipErrorInvalidValue;
    }
}

}  // namespace cavi
