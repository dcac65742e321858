// Tiled, screened E-step + statistics kernel for the common shapes (G in
// {16, 32, 48, 64, 96, 128}, K <= 16).  Same arithmetic as k_estep_stats
// (row log-likelihood l_nk = c_k - sum_g (h_kg x_ng + q_kg)^2, log-sum-exp,
// responsibilities below exp(-87) of the normaliser set to zero, statistics
// around the FP32 centre m_kg), organised for gfx950 and for the sparsity of
// the responsibilities.
//
// Per 2048-row chunk (the unit of the deterministic reduction), 128-row tiles;
// wave w owns rows 32w..32w+31 of every tile and works on them alone (no
// workgroup barrier inside the tile loop): it stages them in its slab of the
// LDS tile (row stride G+4 floats) while the next slab is prefetched into
// registers.  Per slab:
//   A. Screen.  Lane (row j, half) forms, over the first GB genes (16, or 8
//      when K is above 8), the partial sums P_nk of subpopulations half, half+2, ...  Every
//      term is non-negative, so U_nk = c_k - P_nk bounds l_nk from above (also
//      in FP32: adding non-negative terms never lowers a rounded sum).
//      Coefficients are LDS broadcasts from the chunk's (h, q) table.
//   B. Exact terms.  Two lanes per row (each sums half of the remaining genes).
//      First the subpopulation with the largest bound, then every k whose
//      bound is within 87 of that exact value.  A k outside that set has
//      l_nk - L_n < -87, so its responsibility is zero exactly as in the dense
//      computation.  Then log-sum-exp over the computed set: responsibilities,
//      entropy, counts, and a bitmask of nonzero r_nk.
//   C. Statistics.  The same wave walks its rows with lanes over genes; a
//      row with one responsibility of exactly 1 (the common case) adds d and
//      d^2 to its subpopulation's sums, other rows add r d and r d^2 for each
//      nonzero r (d = x - m_kg).
// Each wave sums its rows of a chunk in FP32 (around the previous mean, so
// without cancellation); the four wave sums are promoted to FP64 and added in
// wave order; the chunk partial is written as T0 | T1 | T2 | H.  The chunk's
// first tile is requested before its coefficients are read, and the next tile
// is requested as soon as the current one is in LDS.
#include <math.h>

#include "cavi_impl.h"

namespace cavi {

namespace {

constexpr int kT = 128;  // rows per tile
constexpr uint32_t kOneHot = 1u << 31;
// s_waitcnt immediate for vmcnt(0) with the other counters left alone (gfx9 encoding:
// vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt_hi[15:14])
constexpr int kWaitVm0 = 0x0F70;
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

template <int KT, int G>
struct Cfg {
    static constexpr int XS = G + 4;                     // LDS row stride of the x tile
    static constexpr int LS = (KT == 4) ? 12 : KT + 4;   // LDS row stride of the partial / exact l
    static constexpr int PS = 2 * G + 4;                 // LDS row stride of the (h, q) table
    static constexpr int KH = KT / 2;                    // subpopulations per lane (screen)
    static constexpr int GS = (G + 63) / 64;             // genes per lane (statistics): GS l .. GS l + GS - 1
    static constexpr int LOADS = G / 8;                  // 16-byte loads per lane per 32-row slab
    // screened genes: 16, or 8 for KT = 16 (K above 8), where screening every subpopulation
    // over 16 genes costs more than the exact terms of the extra candidates that 8 let through
    static constexpr int GB = KT > 8 ? 8 : (G < 16 ? G : 16);
    static constexpr int HG = (G - GB) / 2;              // remaining genes per half row
    static constexpr int LDS_BYTES = (kT * XS + kT * LS + KT * PS + KT + KT * G) * 4;
    // waves per SIMD that the LDS allows (160 KB per CU, four waves per workgroup, one per
    // SIMD), 2 or 3: the register-light schedule is built to fit that many (168 registers
    // for 3; a budget of 128 for 4 would spill)
    static constexpr int LDS_WAVES = (163840 / LDS_BYTES) >= 3 ? 3 : 2;
    static_assert(G % 4 == 0 && HG % 4 == 0, "gene blocks of 4");
    static_assert(G % 8 == 0, "a slab must split evenly into 16-byte loads");
    static_assert(8 * KT * G <= kT * XS, "per-wave sums must fit the x tile");
    static_assert(2 * (4 * KT + 4) <= kT * LS, "per-wave counts must fit the l area");
};

// One wave's 32-row slab of a tile.  Its nr rows are contiguous in memory (nr G floats from
// xrow); lane l reads the 16-byte pieces l, l + 64, ... of it.  Pieces past the end of a
// ragged slab re-read its last piece: the loads stay unconditional, so the compiler keeps all
// of them in flight at once, and the offsets are 32-bit from a uniform base.
template <int G, bool OPAQUE>
__device__ __forceinline__ void load_slab(f4 (&pre)[G / 8], const float *__restrict__ xrow, int nr, int lane)
{
    constexpr int C4 = G / 4;
    // OPAQUE: an opaque copy of the lane index, so that the offsets below are recomputed at
    // every call instead of being hoisted out of the tile loop and held for its duration
    int ln = lane;
    if (OPAQUE) asm volatile("" : "+v"(ln));
    const unsigned last = (unsigned)(nr * C4 - 1);
#pragma unroll
    for (int j = 0; j < G / 8; ++j) {
        const unsigned i = min((unsigned)(ln + j * 64), last);
        pre[j] = *(const f4 *)(xrow + 4 * i);
    }
}

// Piece i of the slab belongs to row i / C4 of the wave's LDS slab (row stride G + 4): at
// float offset 4 i + 4 row.  Every piece is stored; rows past a ragged end hold copies of the
// last piece and are never read as data.
template <int G, bool OPAQUE>
__device__ __forceinline__ void store_slab(const f4 (&pre)[G / 8], float *xs, int lane)
{
    constexpr int C4 = G / 4;
    int ln = lane;
    if (OPAQUE) asm volatile("" : "+v"(ln));
#pragma unroll
    for (int j = 0; j < G / 8; ++j) {
        const int i = ln + j * 64;
        const int row = i / C4;
        *(f4 *)(xs + 4 * (i + row)) = pre[j];
    }
}

// the GS consecutive genes of a statistics lane from an LDS row (one 4- or 8-byte read)
template <int GS>
__device__ __forceinline__ void read_genes(float (&v)[GS], const float *p)
{
    static_assert(GS == 1 || GS == 2, "one or two genes per lane");
    if constexpr (GS == 2) {
        const float2 t = *(const float2 *)p;
        v[0] = t.x;
        v[1] = t.y;
    } else {
        v[0] = *p;
    }
}

// m with bit j cleared (one scalar instruction)
__device__ __forceinline__ uint64_t clear_bit(uint64_t m, int j)
{
    asm("s_bitset0_b64 %0, %1" : "+s"(m) : "s"(j));
    return m;
}

// Statistics of Q rows taken in increasing order from the row mask m (which holds at least Q;
// they are cleared from it): u1 += w d, u2 += w d^2 with d = x - centre, row after row, and
// w = 1 without a multiplication when ONE.  All Q LDS reads are issued before the first use.
template <int Q, int GS, int XS, bool ONE, typename WF>
__device__ __forceinline__ void add_rows(uint64_t &m, const float *xl, const float (&mfv)[GS], float (&u1)[GS],
                                         float (&u2)[GS], float &u0, WF weight)
{
    int jr[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        jr[q] = __builtin_ctzll(m);
        m = clear_bit(m, jr[q]);
    }
    float xq[Q][GS], wq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        read_genes<GS>(xq[q], xl + jr[q] * XS);
        wq[q] = ONE ? 1.f : weight(jr[q]);
    }
    if (!ONE) {
#pragma unroll
        for (int q = 0; q < Q; ++q) u0 += wq[q];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int sl = 0; sl < GS; ++sl) {
            const float d = xq[q][sl] - mfv[sl];
            if (ONE) {
                u1[sl] += d;
                u2[sl] = fmaf(d, d, u2[sl]);
            } else {
                const float wv = wq[q] * d;
                u1[sl] += wv;
                u2[sl] = fmaf(wv, d, u2[sl]);
            }
        }
}

// every row of the mask m, four at a time, then two, then one
template <int GS, int XS, bool ONE, typename WF>
__device__ __forceinline__ void add_all_rows(uint64_t m, const float *xl, const float (&mfv)[GS], float (&u1)[GS],
                                             float (&u2)[GS], float &u0, WF weight)
{
    int n = __builtin_popcountll(m);
    for (; n >= 4; n -= 4) add_rows<4, GS, XS, ONE>(m, xl, mfv, u1, u2, u0, weight);
    if (n >= 2) {
        add_rows<2, GS, XS, ONE>(m, xl, mfv, u1, u2, u0, weight);
        n -= 2;
    }
    if (n) add_rows<1, GS, XS, ONE>(m, xl, mfv, u1, u2, u0, weight);
}

// sum over N genes from g0 of (h x + q)^2, x from an LDS row, (h, q) from an LDS table row;
// UNROLL: all loads issued up front (more registers) or one block of 4 genes at a time
template <int N, bool UNROLL>
__device__ __forceinline__ float tail_sum(const float *xr, const float *pr, int g0)
{
    float s = 0.f;
    auto step = [&](int g) {
        const f4 xv = *(const f4 *)(xr + g0 + g);
        const f4 p0 = *(const f4 *)(pr + 2 * (g0 + g));
        const f4 p1 = *(const f4 *)(pr + 2 * (g0 + g) + 4);
        float u;
        u = fmaf(xv.x, p0.x, p0.y); s = fmaf(u, u, s);
        u = fmaf(xv.y, p0.z, p0.w); s = fmaf(u, u, s);
        u = fmaf(xv.z, p1.x, p1.y); s = fmaf(u, u, s);
        u = fmaf(xv.w, p1.z, p1.w); s = fmaf(u, u, s);
    };
    if (UNROLL) {
#pragma unroll
        for (int g = 0; g < N; g += 4) step(g);
    } else {
#pragma unroll 1
        for (int g = 0; g < N; g += 4) step(g);
    }
    return s;
}

// Workgroup barrier that waits only for this wave's LDS operations: the
// prefetch of the next tile (global loads) stays in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The wave's own LDS writes are complete (its lanes exchange data through LDS).
__device__ __forceinline__ void wave_lds_sync()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// partial sum of (h x + q)^2 over the first GB genes of an LDS row for one subpopulation, in the
// screen's order (blocks of 4 genes, fused multiply-adds), so that the exact terms built on it are
// bitwise those of the vector screen
template <int GB>
__device__ __forceinline__ float head_sum(const float *xr, const float *pr)
{
    float acc = 0.f;
#pragma unroll
    for (int gb = 0; gb < GB; gb += 4) {
        const f4 v = *(const f4 *)(xr + gb);
        const float *p = pr + 2 * gb;
        float u;
        u = fmaf(v.x, p[0], p[1]); acc = fmaf(u, u, acc);
        u = fmaf(v.y, p[2], p[3]); acc = fmaf(u, u, acc);
        u = fmaf(v.z, p[4], p[5]); acc = fmaf(u, u, acc);
        u = fmaf(v.w, p[6], p[7]); acc = fmaf(u, u, acc);
    }
    return acc;
}

// maximum over the 16 lanes of a DPP row (lanes 16 q .. 16 q + 15), in every lane of the row
__device__ __forceinline__ float row16_max(float v)
{
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xF, 0xF, false)));  // ror 8
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xF, 0xF, false)));  // ror 4
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x122, 0xF, 0xF, false)));  // ror 2
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x121, 0xF, 0xF, false)));  // ror 1
    return v;
}

}  // namespace

// SCHED: 0 register-heavy, 1 register-light, 2 register-light with the screen as a matrix product
// (BF16 MFMA, subpopulations 9..16): every schedule gives bitwise the same results.
template <int KT, int G, bool INIT, int SCHED>
__global__ __launch_bounds__(kBlock, (SCHED == 1 ? Cfg<KT, G>::LDS_WAVES : 2)) void k_estep_tiled(Shape s, Bufs bf)
{
    constexpr bool LOWREG = SCHED != 0;
    constexpr bool MSCR = SCHED == 2;
    static_assert(!MSCR || (!INIT && KT == 16 && G % 16 == 0), "matrix screen: 16 subpopulation slots, G a multiple of 16");
    using C = Cfg<KT, G>;
    constexpr int XS = C::XS, LS = C::LS, PS = C::PS, KH = C::KH, GS = C::GS, GB = C::GB, HG = C::HG;
    extern __shared__ __align__(16) float smem[];
    float *xs = smem;                 // kT x XS   x tile
    float *ls = xs + kT * XS;         // kT x LS   partial, then exact, row log-likelihood sums
    float *pt = ls + kT * LS;         // KT x PS   (h, q) table
    float *ccs = pt + KT * PS;        // KT        c_k
    float *mft = ccs + KT;            // KT x G   FP32 centres of the statistics

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int jl = lane & 31, half = lane >> 5;
    const float *__restrict__ x = bf.x;

    const int nact = n_active_chunks(s, bf);
    for (int slot = blockIdx.x; slot < nact; slot += gridDim.x) {
        const int chunk = active_chunk(s, bf, slot);
        const int bi = bf.chunk_ds[chunk];
        const Ds d = bf.ds[bi];
        if (!INIT && sweep_skipped(bf.ctl + bi)) continue;
        const int K = d.K, KG = K * G;
        // the chunk's first tile is requested before anything else is read
        const int64_t r0 = d.row0 + (int64_t)(chunk - d.chunk0) * kChunkRows;
        const int nrc = (int)min((int64_t)kChunkRows, (int64_t)d.N - (int64_t)(chunk - d.chunk0) * kChunkRows);
        const int ntiles = (nrc + kT - 1) / kT;
        const int jbase = 32 * w;  // the wave's rows of every tile
        f4 pre[C::LOADS];
        {
            const int nj0 = min(32, min(kT, nrc) - jbase);
            if (nj0 > 0) load_slab<G, LOWREG>(pre, x + (r0 + jbase) * G, nj0, lane);
        }
        const size_t kb = (size_t)bi * s.Kmax;
        const float *__restrict__ cc = bf.cc + kb;
        const float *__restrict__ hq = bf.hq + 2 * kb * G;
        const float *__restrict__ mf = bf.mf + kb * G;
        const float *__restrict__ seedp = bf.seeds + kb * G;
        double *__restrict__ partials = bf.partials;

        // coefficients: every load unconditional (indexes clamped into the dataset's arrays),
        // then one wait, so that no load of the tile loop's prefetch is ever waited on early
        constexpr int NPT = (KT * G + kBlock - 1) / kBlock;
        float hv[NPT], qv[NPT], mv[NPT];
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int ic = min(tid + u * kBlock, KG - 1);
            // initialisation: the table holds the seed rows instead of (h, q)
            hv[u] = INIT ? seedp[ic] : hq[2 * ic];
            qv[u] = INIT ? 0.f : hq[2 * ic + 1];
            mv[u] = mf[ic];
        }
        const float ccv = cc[min(tid, K - 1)];
        // statistics lanes: lane l owns genes GS l .. GS l + GS - 1 when GS l < G; the other
        // lanes read gene 0 onwards instead and their sums are never written
        const bool gown = GS * lane < G;
        const int g0 = gown ? GS * lane : 0;
        // register-heavy schedule: the centres stay in registers for the whole chunk
        float mfr[KT][GS];
#pragma unroll
        for (int k = 0; k < KT; ++k)
#pragma unroll
            for (int sl = 0; sl < GS; ++sl)
                mfr[k][sl] = LOWREG ? 0.f : mf[min(k, K - 1) * G + g0 + sl];
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int i = tid + u * kBlock;
            if (i < KT * G) {
                const int k = i / G, g = i - k * G;
                pt[k * PS + 2 * g] = k < K ? hv[u] : 0.f;
                pt[k * PS + 2 * g + 1] = k < K ? qv[u] : 0.f;
                mft[i] = k < K ? mv[u] : 0.f;
            }
        }
        if (tid < KT) ccs[tid] = tid < K ? ccv : 0.f;
        lds_barrier();  // the coefficient tables are complete
#pragma unroll
        for (int k = 0; k < KT; ++k)
#pragma unroll
            for (int sl = 0; sl < GS; ++sl)
                if (k >= K || !gown) mfr[k][sl] = 0.f;

        // matrix screen: with x' = x - mu_g (mu: the prior centre, FP32) and q' = q + h mu_g,
        //   sum_g (h x + q)^2 = sum_g [h^2 x'^2 + 2 h q' x'] + sum_g q'^2,
        // a product of the rows [x'^2, x'] (BF16) with the coefficients [h^2, 2 h q'] (BF16) on the
        // matrix cores.  Lane l gives the coefficients of subpopulation l % 16 for genes
        // 16 s + 4 (l / 16) + e, e < 4 (step s), and the same genes of its row.
        constexpr int NS = G / 16;
        float mu4[MSCR ? NS : 1][4];
        bf16x8 cf[MSCR ? NS : 1], cfm[MSCR ? NS : 1];
        float cpk = 0.f, e0k = 0.f;
        if constexpr (MSCR) {
            const int kq = lane & 15, q4 = 4 * (lane >> 4);
            float sq = 0.f, wk = 0.f;
#pragma unroll
            for (int st = 0; st < NS; ++st) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int g = 16 * st + q4 + e;
                    const float mu = (float)bf.m0[(size_t)bi * G + g];
                    mu4[st][e] = mu;
                    const float h = pt[kq * PS + 2 * g], qq = pt[kq * PS + 2 * g + 1];
                    const float qp = fmaf(h, mu, qq);
                    const __bf16 a = (__bf16)(h * h), bb = (__bf16)(2.f * h * qp);
                    cf[st][2 * e] = a;
                    cf[st][2 * e + 1] = bb;
                    cfm[st][2 * e] = a;
                    cfm[st][2 * e + 1] = __builtin_bit_cast(__bf16, (unsigned short)(__builtin_bit_cast(unsigned short, bb) & 0x7FFFu));
                    sq = fmaf(qp, qp, sq);
                    const float t = fabsf(qq) + fabsf(h * mu);
                    wk = fmaf(t, t, wk);
                }
            }
            // the four lanes of a subpopulation hold disjoint genes: add their sums
            sq += __shfl_xor(sq, 16, 64);
            sq += __shfl_xor(sq, 32, 64);
            wk += __shfl_xor(wk, 16, 64);
            wk += __shfl_xor(wk, 32, 64);
            // approximate l = (c - sum q'^2) - D, within e0k + 2^-7 |D|m of the exact FP32 l, where
            // |D|m is the same product with |2 h q'| and |x'| (the BF16 roundings of both operands,
            // 2^-8 of each term, dominate; the constant part covers the FP32 roundings)
            cpk = kq < K ? ccs[kq] - sq : -INFINITY;
            e0k = kq < K ? 0x1p-14f * (fabsf(ccs[kq]) + sq + wk + 4.f * G) : 0.f;
        }

        // t0n, t0: the wave's count of one-hot rows and sum of the other responsibilities of
        // subpopulation `lane`, formed in the statistics walk (the soft sums per slab in FP32,
        // then in FP64); t1, t2: the lane's genes' sums
        uint32_t t0n = 0;
        double t0 = 0.0;
        float t1[KT][GS], t2[KT][GS];
#pragma unroll
        for (int k = 0; k < KT; ++k) {
#pragma unroll
            for (int sl = 0; sl < GS; ++sl) t1[k][sl] = t2[k][sl] = 0.f;
        }
        double hacc = 0.0;

        for (int t = 0; t < ntiles; ++t) {
            const int nr = min(kT, nrc - t * kT);
            const int nj = max(0, min(32, nr - jbase));
            // each wave stages, screens, sums and accumulates its own 32 rows: no workgroup
            // barrier inside the tile loop
            if (nj > 0) store_slab<G, LOWREG>(pre, xs + jbase * XS, lane);
            if (t + 1 < ntiles) {
                const int nj1 = min(32, min(kT, nrc - (t + 1) * kT) - jbase);
                if (nj1 > 0) load_slab<G, LOWREG>(pre, x + (r0 + (int64_t)(t + 1) * kT + jbase) * G, nj1, lane);
            }
            wave_lds_sync();
            if (nj == 0) continue;
            const int j = jbase + jl;
            const bool act = jl < nj;

            float rv[KT];
            uint32_t mk = 0;
#pragma unroll
            for (int k = 0; k < KT; ++k) rv[k] = 0.f;
            if (INIT) {
                // hard nearest seed, found by the k-means++ distance passes (FP64 squared
                // distances, genes added in order, the first minimum over the seeds)
                if (act && half == 0) {
                    const uint8_t nb = bf.nearest[r0 + (int64_t)t * kT + j];
                    const int best = nb == kNearestLocked ? 0 : nb;
                    mk = (1u << best) | kOneHot;
                }
            } else {
            if constexpr (MSCR) {
            // A'. matrix screen, two 16-row blocks: lane l takes row 16 blk + l % 16 for the data
            //     and holds l~ of subpopulation l % 16 for rows 16 blk + 4 (l / 16) + v.  Per row:
            //     candidates = {k : l~_k + E_k >= max_j (l~_j - E_j) - 87} (every k with a nonzero
            //     responsibility among them), the first k of largest l~_k - E_k; both written to the
            //     row's slot KT of the l area as (kh << 16) | mask.
            {
                const int kq = lane & 15, qg = lane >> 4;
#pragma unroll
                for (int blk = 0; blk < 2; ++blk) {
                    if (16 * blk >= nj) break;
                    const float *xr0 = xs + (jbase + 16 * blk + kq) * XS + 4 * qg;
                    f32x4_t dd = {0.f, 0.f, 0.f, 0.f}, dm = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int st = 0; st < NS; ++st) {
                        const f4 xv = *(const f4 *)(xr0 + 16 * st);
                        const float p0 = xv.x - mu4[st][0], p1 = xv.y - mu4[st][1];
                        const float p2 = xv.z - mu4[st][2], p3 = xv.w - mu4[st][3];
                        bf16x8 ev;
                        ev[0] = (__bf16)(p0 * p0); ev[1] = (__bf16)p0;
                        ev[2] = (__bf16)(p1 * p1); ev[3] = (__bf16)p1;
                        ev[4] = (__bf16)(p2 * p2); ev[5] = (__bf16)p2;
                        ev[6] = (__bf16)(p3 * p3); ev[7] = (__bf16)p3;
                        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
                        const u32x4 eu = __builtin_bit_cast(u32x4, ev);
                        const bf16x8 em = __builtin_bit_cast(bf16x8, eu & (u32x4){0x7FFFFFFFu, 0x7FFFFFFFu, 0x7FFFFFFFu, 0x7FFFFFFFu});
                        dd = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ev, cf[st], dd, 0, 0, 0);
                        dm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(em, cfm[st], dm, 0, 0, 0);
                    }
                    uint32_t info[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float lt = cpk - dd[v];
                        const float ee = fmaf(0x1p-7f, dm[v], e0k);
                        const float lo = lt - ee, up = lt + ee;
                        const float mlo = row16_max(lo);
                        const uint64_t top = __ballot(lo == mlo);
                        const uint64_t cnd = __ballot(up >= mlo - kLogRCut);
                        const uint32_t tb = (uint32_t)(top >> (16 * qg)) & 0xFFFFu;
                        const uint32_t cb = (uint32_t)(cnd >> (16 * qg)) & 0xFFFFu;
                        // a row without a finite bound (non-finite data) takes subpopulation 0 alone
                        info[v] = tb ? ((uint32_t)__builtin_ctz(tb) << 16) | cb : 0u;
                    }
                    if (kq == 0) {
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            ((uint32_t *)ls)[(jbase + 16 * blk + 4 * qg + v) * LS + KT] = info[v];
                    }
                }
            }
            } else {
            // A. screen: partial sums over the first GB genes; lane (row j, half) takes
            //    subpopulations half, half + 2, ...  Every lane writes all of its slots (a
            //    skipped subpopulation k >= K, or a row past the end, leaves a value that is
            //    never read), so that only the test k < K branches.
            {
                const float *xa = xs + j * XS;
                f4 va[GB / 4];
#pragma unroll
                for (int gb = 0; gb < GB; gb += 4) va[gb / 4] = *(const f4 *)(xa + gb);
#pragma unroll
                for (int i = 0; i < KH; ++i) {
                    const int k = half + 2 * i;
                    float acc = 0.f;
                    if (k < K) {
#pragma unroll
                        for (int gb = 0; gb < GB; gb += 4) {
                            const float *p = pt + k * PS + 2 * gb;
                            const float h0 = p[0], q0 = p[1], h1 = p[2], q1 = p[3];
                            const float h2 = p[4], q2 = p[5], h3 = p[6], q3 = p[7];
                            const f4 v = va[gb / 4];
                            float u;
                            u = fmaf(v.x, h0, q0); acc = fmaf(u, u, acc);
                            u = fmaf(v.y, h1, q1); acc = fmaf(u, u, acc);
                            u = fmaf(v.z, h2, q2); acc = fmaf(u, u, acc);
                            u = fmaf(v.w, h3, q3); acc = fmaf(u, u, acc);
                        }
                    }
                    ls[j * LS + k] = acc;
                }
            }
            }  // screens
            wave_lds_sync();

            // B. exact terms for the candidate subpopulations of row j (lanes jl, jl+32)
            float *lr = ls + j * LS;
            const float *xr = xs + j * XS;
            uint32_t done = 0;
            int kone = 0;      // the best-bounded subpopulation and its exact l
            float lone = 0.f;
            if (GB == G) {
                if (act && half == 0) {
#pragma unroll
                    for (int k = 0; k < KT; ++k)
                        if (k < K) lr[k] = ccs[k] - lr[k];
                }
                done = (1u << K) - 1u;
            } else {
                float U[KT];
                int kh = 0;
                uint32_t cmask = 0;  // matrix screen: the row's candidates
                if constexpr (MSCR) {
                    const uint32_t info = act ? ((const uint32_t *)lr)[KT] : 0u;
                    kh = (int)(info >> 16);
                    cmask = info & 0xFFFFu;
                } else {
                    float best = -INFINITY;
                    // the row's partial sums and the c_k, read whole (16-byte reads, no branches)
                    float lv[KT], cv[KT];
#pragma unroll
                    for (int q = 0; q < KT; q += 4) {
                        const f4 a = *(const f4 *)(lr + q);
                        const f4 c = *(const f4 *)(ccs + q);
                        lv[q] = a.x, lv[q + 1] = a.y, lv[q + 2] = a.z, lv[q + 3] = a.w;
                        cv[q] = c.x, cv[q + 1] = c.y, cv[q + 2] = c.z, cv[q + 3] = c.w;
                    }
#pragma unroll
                    for (int k = 0; k < KT; ++k) {
                        U[k] = (k < K && act) ? cv[k] - lv[k] : -INFINITY;
                        if (U[k] > best) {
                            best = U[k];
                            kh = k;
                        }
                    }
                }
                // exact l for the first subpopulation (the best bounded)
                const float pkh = MSCR ? (act ? head_sum<GB>(xr, pt + kh * PS) : 0.f) : lr[kh];
                const float sh = act ? tail_sum<HG, !LOWREG>(xr, pt + kh * PS, GB + half * HG) : 0.f;
                const float so = __shfl_xor(sh, 32, 64);
                const float lkh = ccs[kh] - (pkh + (half == 0 ? sh + so : so + sh));
                kone = kh;
                lone = lkh;
                uint32_t cm = 0;
                if constexpr (MSCR) {
                    cm = cmask & ~(1u << kh);
                } else {
#pragma unroll
                    for (int k = 0; k < KT; ++k)
                        if (k < K && k != kh && U[k] - lkh >= -kLogRCut) cm |= 1u << k;
                }
                if (!act) cm = 0;
                __builtin_amdgcn_wave_barrier();
                if (act && half == 0) lr[kh] = lkh;
                done = 1u << kh;
                // remaining candidates, one per lane per round
                while (__ballot(cm != 0)) {
                    const bool mine = cm != 0;
                    const int k = mine ? __builtin_ctz(cm) : 0;
                    const float pk = MSCR ? (mine ? head_sum<GB>(xr, pt + k * PS) : 0.f) : lr[k];
                    const float sk = mine ? tail_sum<HG, !LOWREG>(xr, pt + k * PS, GB + half * HG) : 0.f;
                    const float sko = __shfl_xor(sk, 32, 64);
                    __builtin_amdgcn_wave_barrier();
                    if (mine) {
                        if (half == 0) lr[k] = ccs[k] - (pk + (sk + sko));
                        done |= 1u << k;
                        cm &= cm - 1u;
                    }
                }
            }
            if (!act) done = 0;
            __builtin_amdgcn_wave_barrier();

            // log-sum-exp over the computed set (lanes jl < 32 own the rows).  When every row
            // of the slab has a single candidate (the usual case for well-separated
            // subpopulations) the exact values are written directly: responsibility 1 and entropy
            // term 0 for a finite l (r = 0 and a NaN entropy otherwise, as in the general form).
            // (Not for KT = 16, where the second form costs more registers than it saves.)
            bool single = false;
            if constexpr (GB < G && KT <= 8) single = !__ballot(act && half == 0 && done != (1u << kone));
            if (single) {
                // every row of the slab is one-hot (or has no finite term): the statistics walk
                // needs no responsibilities, only the row masks
                if (act && half == 0) {
                    const bool fin = isfinite(lone);
                    if (fin) mk |= (1u << kone) | kOneHot;
                    hacc += fin ? 0.0 : (double)__int_as_float(0x7fc00000);
                }
            } else if (KT > 8 && act) {
                // the row's two lanes share the subpopulations: half h forms those of
                // KT/2 h .. KT/2 h + KT/2 - 1 and the halves exchange maximum, sum, entropy,
                // counts and masks; the responsibilities replace the row's l values in LDS
                constexpr int KQ = KT / 2;
                const int kb = half * KQ;
                float l[KQ];
#pragma unroll
                for (int q = 0; q < KQ; q += 4) {
                    const f4 a = *(const f4 *)(lr + kb + q);
                    l[q] = a.x, l[q + 1] = a.y, l[q + 2] = a.z, l[q + 3] = a.w;
                }
                const uint32_t dh = done >> kb;
#pragma unroll
                for (int j = 0; j < KQ; ++j) l[j] = (dh & (1u << j)) ? l[j] : -INFINITY;
                float mxh = l[0];
#pragma unroll
                for (int j = 1; j < KQ; ++j) mxh = fmaxf(mxh, l[j]);
                const float mx = fmaxf(mxh, __shfl_xor(mxh, 32, 64));
                float seh = 0.f;
#pragma unroll
                for (int j = 0; j < KQ; ++j) {
                    const float e = __expf(l[j] - mx);
                    seh += (dh & (1u << j)) ? e : 0.f;
                }
                const float se = seh + __shfl_xor(seh, 32, 64);
                const float L = mx + __logf(se);
                float hh = (half == 0 && !isfinite(L)) ? __int_as_float(0x7fc00000) : 0.f;
                int nzh = 0;
                uint32_t mkh = 0;
                float rsum = 0.f, rq[KQ];
#pragma unroll
                for (int j = 0; j < KQ; ++j) {
                    const float dl = l[j] - L;
                    const bool take = (dh & (1u << j)) && dl > -kLogRCut;
                    const float e = __expf(dl);
                    rq[j] = take ? e : 0.f;
                    hh = take ? hh - rq[j] * dl : hh;
                    mkh |= rq[j] != 0.f ? 1u << (kb + j) : 0u;
                    nzh += rq[j] != 0.f;
                    rsum += rq[j];
                }
                const int nz = nzh + __shfl_xor(nzh, 32, 64);
                // with a single nonzero term the sum is that term, whatever the order
                const float rone = rsum + __shfl_xor(rsum, 32, 64);
                const uint32_t mka = mkh | (uint32_t)__shfl_xor((int)mkh, 32, 64);
                const float h = hh + __shfl_xor(hh, 32, 64);
                if (half == 0) {
                    mk |= mka;
                    if (nz == 1 && rone == 1.f) mk |= kOneHot;
                    hacc += (double)h;
                }
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int q = 0; q < KQ; q += 4) *(f4 *)(lr + kb + q) = f4{rq[q], rq[q + 1], rq[q + 2], rq[q + 3]};
            } else if (KT <= 8 && act && half == 0) {
                // every term is formed and the computed set selects it (no branches); adding
                // +0 for a term outside the set leaves a sum unchanged
                float l[KT];
#pragma unroll
                for (int q = 0; q < KT; q += 4) {
                    const f4 a = *(const f4 *)(lr + q);
                    l[q] = a.x, l[q + 1] = a.y, l[q + 2] = a.z, l[q + 3] = a.w;
                }
#pragma unroll
                for (int k = 0; k < KT; ++k) l[k] = (done & (1u << k)) ? l[k] : -INFINITY;
                float mx = l[0];
#pragma unroll
                for (int k = 1; k < KT; ++k) mx = fmaxf(mx, l[k]);
                float se = 0.f;
#pragma unroll
                for (int k = 0; k < KT; ++k) {
                    const float e = __expf(l[k] - mx);
                    se += (done & (1u << k)) ? e : 0.f;
                }
                const float L = mx + __logf(se);
                float h = isfinite(L) ? 0.f : __int_as_float(0x7fc00000);
                int nz = 0;
#pragma unroll
                for (int k = 0; k < KT; ++k) {
                    const float dl = l[k] - L;
                    const bool take = (done & (1u << k)) && dl > -kLogRCut;
                    const float e = __expf(dl);
                    rv[k] = take ? e : 0.f;
                    h = take ? h - rv[k] * dl : h;
                    mk |= rv[k] != 0.f ? 1u << k : 0u;
                    nz += rv[k] != 0.f;
                }
                if (nz == 1) {
                    float rone = 0.f;
#pragma unroll
                    for (int k = 0; k < KT; ++k) rone += rv[k];
                    if (rone == 1.f) mk |= kOneHot;
                }
                hacc += (double)h;
                if (LOWREG) {
                    // the responsibilities replace the row's l values in LDS for the statistics
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int q = 0; q < KT; q += 4) *(f4 *)(lr + q) = f4{rv[q], rv[q + 1], rv[q + 2], rv[q + 3]};
                }
            }
            if (LOWREG || KT > 8) wave_lds_sync();

            }  // phases A, B and log-sum-exp

            // C. statistics over the same rows, lanes over genes.  For each subpopulation
            //    walk the rows whose responsibility for it is nonzero, four rows per step so
            //    that their LDS reads overlap; rows with a single responsibility of exactly 1
            //    skip the multiplication.  Rows are added one after another in increasing
            //    order (one-hot rows first).  With KT = 16 the subpopulation loop is not unrolled, so the sums
            //    cannot be indexed statically: the slab's rows are summed in two registers
            //    and that sum is added to the wave's running sum; otherwise the rows are
            //    added to the running sum directly.
            if (nj > 0) {
                // the lane's first gene, as an opaque value in the register-light schedule: the
                // LDS addresses below are formed from it here rather than hoisted out of the
                // tile loop and held
                int gq = g0;
                if (LOWREG) asm volatile("" : "+v"(gq));
                const float *xl = xs + jbase * XS + gq;
                constexpr bool kSlabSums = KT > 8;
                // mk is zero outside the rows this wave owns
                const uint64_t hard = __ballot(mk & kOneHot);
#pragma unroll
                for (int k = 0; k < KT; ++k) {
                    if (k >= K) break;
                    const uint64_t rows = __ballot((mk >> k) & 1u);
                    if (!rows) continue;
                    const uint64_t one = rows & hard;
                    const uint64_t soft = rows & ~hard;
                    float mfv[GS], u1[GS], u2[GS];
#pragma unroll
                    for (int sl = 0; sl < GS; ++sl) {
                        u1[sl] = kSlabSums ? 0.f : t1[k][sl];
                        u2[sl] = kSlabSums ? 0.f : t2[k][sl];
                    }
                    if (LOWREG) {
                        read_genes<GS>(mfv, mft + k * G + gq);
                    } else {
#pragma unroll
                        for (int sl = 0; sl < GS; ++sl) mfv[sl] = mfr[k][sl];
                    }
                    // counts: the one-hot rows (responsibility exactly 1), then the others' weights
                    // in row order
                    if (lane == k) t0n += (uint32_t)__builtin_popcountll(one);
                    float u0 = 0.f;
                    const auto unit = [](int) { return 1.f; };
                    add_all_rows<GS, XS, true>(one, xl, mfv, u1, u2, u0, unit);
                    if (soft) {
                        const auto resp = [&](int jj) {
                            return (LOWREG || KT > 8)
                                       ? ls[(jbase + jj) * LS + k]
                                       : __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rv[k]), jj));
                        };
                        add_all_rows<GS, XS, false>(soft, xl, mfv, u1, u2, u0, resp);
                        if (lane == k) t0 += (double)u0;
                    }
#pragma unroll
                    for (int sl = 0; sl < GS; ++sl) {
                        t1[k][sl] = kSlabSums ? t1[k][sl] + u1[sl] : u1[sl];
                        t2[k][sl] = kSlabSums ? t2[k][sl] + u2[sl] : u2[sl];
                    }
                }
            }
        }
        lds_barrier();  // every wave is done with its rows

        // combine the four waves in wave order: every wave leaves its FP32 sums in the LDS of
        // the x tile (and its FP64 count and entropy sums in the l area); each chunk statistic
        // is then ((w0 + w1) + w2) + w3 in FP64
        float *ws = xs;              // 4 x 2KG
        double *wd = (double *)ls;   // 4 x KT counts, then 4 entropies
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            if (k < K) {
                if (lane == k) wd[w * KT + k] = (double)t0n + t0;
                if (gown) {
#pragma unroll
                    for (int sl = 0; sl < GS; ++sl) {
                        ws[w * 2 * KG + k * G + g0 + sl] = t1[k][sl];
                        ws[w * 2 * KG + KG + k * G + g0 + sl] = t2[k][sl];
                    }
                }
            }
        }
        const double hw = wave_sum(hacc);
        if (lane == 0) wd[4 * KT + w] = hw;
        lds_barrier();
        double *out = partials + (size_t)chunk * s.Smax;
        for (int i = tid; i < K + 2 * KG + 1; i += kBlock) {
            double v;
            if (i < K) {
                v = ((wd[i] + wd[KT + i]) + wd[2 * KT + i]) + wd[3 * KT + i];
            } else if (i < K + 2 * KG) {
                const int j = i - K;
                v = (((double)ws[j] + (double)ws[2 * KG + j]) + (double)ws[4 * KG + j]) + (double)ws[6 * KG + j];
            } else {
                v = ((wd[4 * KT] + wd[4 * KT + 1]) + wd[4 * KT + 2]) + wd[4 * KT + 3];
            }
            out[i] = v;
        }
        lds_barrier();
    }
}

namespace {

template <int KT, int G>
hipError_t launch_t(const Shape &s, const Bufs &b, int init_mode, hipStream_t st)
{
    constexpr int lds = Cfg<KT, G>::LDS_BYTES;
    if (init_mode)
        hipLaunchKernelGGL((k_estep_tiled<KT, G, true, 1>), dim3(s.egrid), dim3(kBlock), lds, st, s, b);
    else if constexpr (KT == 16 && G % 16 == 0) {
        if (s.schedule == 2)
            hipLaunchKernelGGL((k_estep_tiled<KT, G, false, 2>), dim3(s.egrid), dim3(kBlock), lds, st, s, b);
        else if (s.schedule == 1)
            hipLaunchKernelGGL((k_estep_tiled<KT, G, false, 1>), dim3(s.egrid), dim3(kBlock), lds, st, s, b);
        else
            hipLaunchKernelGGL((k_estep_tiled<KT, G, false, 0>), dim3(s.egrid), dim3(kBlock), lds, st, s, b);
    } else if (s.schedule == 1)
        hipLaunchKernelGGL((k_estep_tiled<KT, G, false, 1>), dim3(s.egrid), dim3(kBlock), lds, st, s, b);
    else
        hipLaunchKernelGGL((k_estep_tiled<KT, G, false, 0>), dim3(s.egrid), dim3(kBlock), lds, st, s, b);
    return hipGetLastError();
}

template <int KT>
hipError_t launch_g(const Shape &s, const Bufs &b, int init_mode, hipStream_t st)
{
    switch (s.G) {
    case 16: return launch_t<KT, 16>(s, b, init_mode, st);
    case 32: return launch_t<KT, 32>(s, b, init_mode, st);
    case 48: return launch_t<KT, 48>(s, b, init_mode, st);
    case 64: return launch_t<KT, 64>(s, b, init_mode, st);
    case 96: return launch_t<KT, 96>(s, b, init_mode, st);
    case 128: return launch_t<KT, 128>(s, b, init_mode, st);
    default: return hipErrorInvalidValue;
    }
}

int lds_bytes(int kt, int G)
{
    const int ls = (kt == 4) ? 12 : kt + 4;
    return (kT * (G + 4) + kT * ls + kt * (2 * G + 4) + kt) * 4 + kBlock * 8;
}

}  // namespace

bool tiled_supported(int K, int G)
{
    const bool g_ok = G == 16 || G == 32 || G == 48 || G == 64 || G == 96 || G == 128;
    if (!g_ok) return false;
    const int kt = choose_kt(K);
    const int gs = (G + 63) / 64;
    if (kt > 16 || kt * gs > 16) return false;
    return lds_bytes(kt, G) <= (g_lds_limit > 0 ? g_lds_limit : 65536);
}

hipError_t launch_estep_tiled(const Shape &s, const Bufs &b, int init_mode, hipStream_t st)
{
    switch (s.kt) {
    case 4: return launch_g<4>(s, b, init_mode, st);
    case 8: return launch_g<8>(s, b, init_mode, st);
    case 16:
        switch (s.G) {
        case 16: return launch_t<16, 16>(s, b, init_mode, st);
        case 32: return launch_t<16, 32>(s, b, init_mode, st);
        case 48: return launch_t<16, 48>(s, b, init_mode, st);
        case 64: return launch_t<16, 64>(s, b, init_mode, st);
        default: return hipErrorInvalidValue;
        }
    default: return hipErrorInvalidValue;
    }
}

}  // namespace cavi
