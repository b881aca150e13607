// Backward (adjoint) kernels of the APH predistorter for gfx950.
//
// The forward map of Eq. (1), written with s = |x|^2, v = (Re x, Im x) and the
// precombined real 2x2 matrices M_{j,k} (order 2j+1, tap k), is
//     z_n = c + sum_k sum_j M_{j,k} s_{n-k}^j v_{n-k}.
// For a real loss E with G_n = dE/dRe z_n + j dE/dIm z_n (as a real 2-vector):
//   coefficients:  dE/dM_{j,k}[r][c] = sum_m G_{m+k}[r] * (s_m^j v_m)[c],
//                  dE/dc = sum_n G_n;
//   inputs:        dE/dv_m = sum_j [ s^j U_j + 2 j s^(j-1) v (v . U_j) ],
//                  U_j(m) = sum_k M_{j,k}^T G_{m+k}   (G_n = 0 for n >= N),
// i.e. the transpose of the filter (a correlation with the taps) followed by
// the transposed Jacobian of the pointwise basis.  The basis is recomputed
// from x; nothing from the forward pass is stored.  The chain rule through
// M = [[hr+gr, gi-hi], [hi+gi, hr-gr]] to the coefficients of the paper's
// stacking happens in the FP64 finalisation kernel.
//
// Reduction of the coefficient gradient is deterministic: each lane sums its
// own samples in a fixed order (FP32, at most kBwdFlush chunks at a time), the
// wave reduces those sums in a fixed tree into its FP64 totals, the block adds
// its waves' totals in order, one partial per block goes to the workspace, and
// a single block sums the partials in FP64 in block order.
#pragma once

#include "dpd_fwd_kernels.h"
#include "dpd_reduce.h"

namespace dpd {

struct BwdParams {
    const float2 *x;
    const float2 *gz;
    float2 *gx;           // nullptr: no input gradient
    float *partials;      // [gridDim.x][E] (E = 4*L*NI + 2), nullptr: no coeff gradient
    int64_t n, ld, rows;
    int64_t tpr;          // full chunks per row (n / (64*S)); the ragged end is extra
    const float *M;       // precombined table
};

typedef hipError_t (*BwdLaunch)(const BwdParams &, hipStream_t, int grid);

struct BwdTable {
    BwdLaunch fn[kSpecNI][kSpecL][3];   // [.][.][want: 0 = dx, 1 = dcoef, 2 = both]
    const void *kern[kSpecNI][kSpecL][3];
};

void register_bwd_ni1(BwdTable &);
void register_bwd_ni2(BwdTable &);
void register_bwd_ni3(BwdTable &);
void register_bwd_ni4(BwdTable &);
void register_bwd_ni5(BwdTable &);
void register_bwd_ni6(BwdTable &);
void register_bwd_ni7(BwdTable &);
void register_bwd_ni8(BwdTable &);

constexpr int kBwdS = 4;   // consecutive samples per lane
// Chunks a lane's FP32 coefficient-gradient sums cover before they are added
// to the wave's FP64 totals (a power of two): 32 chunks = 128 samples per lane.
constexpr int kBwdFlush = 32;

// FP64 sums of table entry q's four coefficient-gradient partials (two for
// q = L NI, the c entry) over nblk blocks: each thread its strided share of
// the blocks in order, then the DPP lane sum of each wave and the four waves
// in order (bitwise reproducible).  u is valid in thread 0.
__device__ __forceinline__ void dcoef_block_sums(const float *__restrict__ partials, int nblk, const CoefMap &map,
                                                 int q, double (&red)[kBlock / 64][4], double (&u)[4])
{
    const int E = 4 * map.L * map.NI + 2;
    const bool dc = q == map.L * map.NI;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        const float *pp = partials + (int64_t)b * E + 4 * q;
        a[0] += (double)pp[0];
        a[1] += (double)pp[1];
        if (!dc) {
            a[2] += (double)pp[2];
            a[3] += (double)pp[3];
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        a[e] = wave_sum_to_lane63(a[e]);
        if (lane == 63) red[wv][e] = a[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        u[e] = red[0][e];
        for (int w = 1; w < kBlock / 64; ++w) u[e] += red[w][e];
    }
}

// The chain rule from table entry q's sums to the coefficients of the
// section 2.2 stacking (M = [[hr+gr, gi-hi], [hi+gi, hr-gr]], order 2j+1,
// tap k): u1 = dE/dm00, u4 = dE/dm01, u3 = dE/dm10, u2 = dE/dm11,
//   grad h = (u1 + u2) + j (u3 - u4),  grad hbar = (u1 - u2) + j (u3 + u4),
//   grad c = sum G (q = L NI).
// Returns how many coefficients (0..2) entry q feeds: idx[i], grad[i].
__device__ __forceinline__ int dcoef_block_grads(const CoefMap &map, int q, const double (&u)[4], int (&idx)[2],
                                                 float2 (&grad)[2])
{
    const int L = map.L, NI = map.NI;
    if (q == L * NI) {
        idx[0] = (map.n_main + map.n_conj) * L;
        grad[0] = make_float2((float)u[0], (float)u[1]);
        return 1;
    }
    const int k = q / NI, j = q - k * NI;
    const double u1 = u[0], u4 = u[1], u3 = u[2], u2 = u[3];
    int c = 0;
    if (map.main_idx[j] >= 0) {
        idx[c] = map.main_idx[j] * L + k;
        grad[c++] = make_float2((float)(u1 + u2), (float)(u3 - u4));
    }
    if (map.conj_idx[j] >= 0) {
        idx[c] = (map.n_main + map.conj_idx[j]) * L + k;
        grad[c++] = make_float2((float)(u1 - u2), (float)(u3 + u4));
    }
    return c;
}

template <bool B>
struct BwdTag {
    static constexpr bool value = B;
};

// Persistent grid over the full chunks (C = 64*S samples) of all rows, wave g
// taking chunks g, g + nw, ... (rows flattened), then the ragged row ends.
// Per chunk the wave stages G (the chunk plus the L-1 samples after it; zero
// past the row end) and x (the chunk) in padded wave-private LDS buffers,
// with nontemporal 1 KiB-contiguous loads issued one chunk ahead: a chunk's
// registers are staged right after the previous chunk's stores, and the next
// chunk's loads go out into the same registers before the staged chunk is
// filtered, so the compiler's counter waits never cover the prefetch.  Each
// lane owns S consecutive samples m and reads G_{m..m+S+L-2}.  One pass over
// the power levels j (ascending) produces both gradients: U_j by taps for dx
// (P = sum s^j U_j and 2Q = sum 2j s^(j-1) v.U_j accumulated with explicit
// powers; dx = P + 2Q v), and G (x) s^j v into the per-lane coefficient
// accumulators.
template <int NI, int L, bool DX, bool DC>
__global__ void __launch_bounds__(kBlock) bwd_kernel(BwdParams p)
{
    constexpr int S = kBwdS;
    constexpr int C = 64 * S;
    constexpr int W = S + L - 1;
    constexpr int NV = S / 2;
    constexpr int WAVES = kBlock / 64;
    constexpr int NM = 4 * L * NI;                              // matrix floats (c has no gradient path here)
    constexpr int E = NM + 2;
    constexpr int HS = L - 1;                                   // right halo
    constexpr int GSLOTS = C + HS + (C + HS) / S + 1;
    constexpr int XSLOTS = C + C / S;
    __shared__ __align__(16) float2 gs[WAVES][GSLOTS];
    __shared__ __align__(16) float2 xsh[WAVES][XSLOTS];
    __shared__ __align__(16) float mt[NM];
    __shared__ double red[DC ? WAVES * E : 1];   // per-wave FP64 totals of the coefficient gradient

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int e = tid; e < NM; e += kBlock) mt[e] = p.M[e];
    __syncthreads();
    float2 *G = gs[wv];
    float2 *X = xsh[wv];
    // slot of chunk-relative sample d: one pad after every S
    auto slot = [](int d) { return d + d / S; };
    const int hl = HS > 0 ? (lane < HS ? lane : HS - 1) : 0;

    float acc[DC ? E : 1];
#pragma unroll
    for (int e = 0; e < (DC ? E : 1); ++e) acc[e] = 0.f;
    // The per-lane FP32 sums cover at most kBwdFlush chunks: then they are
    // summed over the wave and added to the wave's FP64 totals (entry
    // 64 g + l in lane l of tot[g]), so the rounding error does not grow with
    // the stream length.
    constexpr int NGT = DC ? (E + 63) / 64 : 1;
    double tot[NGT];
#pragma unroll
    for (int g = 0; g < NGT; ++g) tot[g] = 0.0;
    auto flush = [&]() {
        if constexpr (DC) {
            wave_sums_into<E>(acc, tot, lane);
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = 0.f;
        }
    };

    struct Regs {
        float4 g[NV];
        float4 x[NV];
        float2 gh;   // raw G_{t0 + C + hl} (replaced by zero past the row end at staging)
    };
    // full chunk at (row, t0): every load unconditional
    auto load_full = [&](Regs &R, int64_t row, int64_t t0) {
        const v4f *g4 = reinterpret_cast<const v4f *>(p.gz + row * p.ld + t0);
        const v4f *x4 = reinterpret_cast<const v4f *>(p.x + row * p.ld + t0);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const v4f u = __builtin_nontemporal_load(g4 + lane + 64 * i);
            R.g[i] = make_float4(u.x, u.y, u.z, u.w);
        }
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const v4f u = __builtin_nontemporal_load(x4 + lane + 64 * i);
            R.x[i] = make_float4(u.x, u.y, u.z, u.w);
        }
        if (HS > 0) {
            const int64_t m = t0 + C + hl;
            R.gh = p.gz[row * p.ld + (m < p.n ? m : p.n - 1)];
        }
    };
    // ragged row end: samples past n read as zero
    auto load_part = [&](Regs &R, int64_t row, int64_t t0) {
        const float2 *gr = p.gz + row * p.ld;
        const float2 *xr = p.x + row * p.ld;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int64_t m = t0 + 2 * (lane + 64 * i);
            const float2 a = m < p.n ? gr[m] : make_float2(0.f, 0.f);
            const float2 b = m + 1 < p.n ? gr[m + 1] : make_float2(0.f, 0.f);
            R.g[i] = make_float4(a.x, a.y, b.x, b.y);
            const float2 c = m < p.n ? xr[m] : make_float2(0.f, 0.f);
            const float2 d = m + 1 < p.n ? xr[m + 1] : make_float2(0.f, 0.f);
            R.x[i] = make_float4(c.x, c.y, d.x, d.y);
        }
        R.gh = make_float2(0.f, 0.f);
    };
    auto stage = [&](const Regs &R, int64_t t0) {
        wave_lds_order();   // the previous chunk's LDS reads are done
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int j = 2 * (lane + 64 * i);
            G[slot(j)] = make_float2(R.g[i].x, R.g[i].y);
            G[slot(j) + 1] = make_float2(R.g[i].z, R.g[i].w);
            X[slot(j)] = make_float2(R.x[i].x, R.x[i].y);
            X[slot(j) + 1] = make_float2(R.x[i].z, R.x[i].w);
        }
        if (HS > 0 && lane < HS) G[slot(C + lane)] = t0 + C + lane < p.n ? R.gh : make_float2(0.f, 0.f);
        wave_lds_order();
    };
    // gradients of a staged chunk; FULL: every sample of it is inside the row
    auto compute = [&](int64_t row, int64_t t0, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        // An opaque zero keeps the table reads inside the loop (hoisted, the
        // whole table would occupy registers next to the accumulators).
        int z = 0;
        asm volatile("" : "+v"(z));
        const float4 *M4 = reinterpret_cast<const float4 *>(mt + z);
        float ga[W], gb[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const float2 g = G[slot(lane * S + w)];
            ga[w] = g.x;
            gb[w] = g.y;
        }
        float va[S], vb[S], sq[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const float2 v = X[slot(lane * S + i)];
            va[i] = v.x;
            vb[i] = v.y;
            sq[i] = __builtin_fmaf(v.x, v.x, v.y * v.y);
        }
        float Pa[S], Pb[S], Q[S], pw[S], pwl[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            Pa[i] = Pb[i] = Q[i] = 0.f;
            pw[i] = 1.f;     // s^j
            pwl[i] = 0.f;    // 2 j s^(j-1)
        }
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            float Ua[S], Ub[S], ba[S], bb[S];
#pragma unroll
            for (int i = 0; i < S; ++i) {
                Ua[i] = Ub[i] = 0.f;
                ba[i] = pw[i] * va[i];
                bb[i] = pw[i] * vb[i];
            }
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const float4 m = M4[k * NI + j];   // [[m.x, m.y], [m.z, m.w]]
#pragma unroll
                for (int i = 0; i < S; ++i) {
                    const float a = ga[i + k], b = gb[i + k];
                    if constexpr (DX) {
                        Ua[i] = __builtin_fmaf(m.x, a, Ua[i]);
                        Ua[i] = __builtin_fmaf(m.z, b, Ua[i]);
                        Ub[i] = __builtin_fmaf(m.y, a, Ub[i]);
                        Ub[i] = __builtin_fmaf(m.w, b, Ub[i]);
                    }
                    if constexpr (DC) {
                        float *u = &acc[4 * (k * NI + j)];
                        u[0] = __builtin_fmaf(a, ba[i], u[0]);
                        u[1] = __builtin_fmaf(a, bb[i], u[1]);
                        u[2] = __builtin_fmaf(b, ba[i], u[2]);
                        u[3] = __builtin_fmaf(b, bb[i], u[3]);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < S; ++i) {
                if constexpr (DX) {
                    // level 0 has s^0 = 1: P starts at U_0
                    Pa[i] = j == 0 ? Ua[i] : __builtin_fmaf(pw[i], Ua[i], Pa[i]);
                    Pb[i] = j == 0 ? Ub[i] : __builtin_fmaf(pw[i], Ub[i], Pb[i]);
                    if (j > 0) {
                        const float d = __builtin_fmaf(va[i], Ua[i], vb[i] * Ub[i]);
                        Q[i] = j == 1 ? pwl[i] * d : __builtin_fmaf(pwl[i], d, Q[i]);
                    }
                    pwl[i] = (float)(2 * (j + 1)) * pw[i];   // 2 (j + 1) s^j: Q carries the factor 2 of dx
                }
                pw[i] *= sq[i];
            }
            // One power level at a time: the empty asm statements consume this
            // level's results, so the instruction selector cannot sink its
            // multiply-adds past the barrier (it did, which kept every
            // level's table entries live at once); only this level's L
            // table entries are in registers.
            if constexpr (DC) {
#pragma unroll
                for (int k = 0; k < L; ++k)
#pragma unroll
                    for (int q = 0; q < 4; ++q) asm volatile("" ::"v"(acc[4 * (k * NI + j) + q]));
            }
            if constexpr (DX) {
#pragma unroll
                for (int i = 0; i < S; ++i) asm volatile("" ::"v"(Pa[i]), "v"(Pb[i]), "v"(Q[i]));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (DC) {
#pragma unroll
            for (int i = 0; i < S; ++i) {
                acc[E - 2] += ga[i];
                acc[E - 1] += gb[i];
            }
        }
        if constexpr (DX) {
            float dxa[S], dxb[S];
#pragma unroll
            for (int i = 0; i < S; ++i) {
                dxa[i] = __builtin_fmaf(Q[i], va[i], Pa[i]);
                dxb[i] = __builtin_fmaf(Q[i], vb[i], Pb[i]);
            }
            float2 *gxr = p.gx + row * p.ld;
            if constexpr (FULL) {
                // back through LDS so every store instruction writes 1 KiB
                wave_lds_order();
#pragma unroll
                for (int i = 0; i < S; ++i) G[slot(lane * S + i)] = make_float2(dxa[i], dxb[i]);
                wave_lds_order();
                v4f *o4 = reinterpret_cast<v4f *>(gxr + t0);
#pragma unroll
                for (int i = 0; i < NV; ++i) {
                    const int j = 2 * (lane + 64 * i);
                    const float2 u = G[slot(j)], w = G[slot(j) + 1];
                    const v4f v = {u.x, u.y, w.x, w.y};
                    __builtin_nontemporal_store(v, o4 + lane + 64 * i);
                }
            } else {
                const int64_t m0 = t0 + (int64_t)lane * S;
#pragma unroll
                for (int i = 0; i < S; ++i)
                    if (m0 + i < p.n) gxr[m0 + i] = make_float2(dxa[i], dxb[i]);
            }
        }
    };

    const int64_t tpr = p.tpr;                   // full chunks per row
    const int64_t total = p.rows * tpr;
    const int64_t nw = (int64_t)gridDim.x * WAVES;
    const int64_t gw = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * WAVES + wv;
    if (gw < total) {
        const int64_t left = (total - 1 - gw) / nw + 1;
        // (row, chunk in row) advanced by nw chunks per step without a division
        const int64_t dq = nw / tpr, dr = nw - dq * tpr;
        int64_t row = gw / tpr, tix = gw - row * tpr;
        Regs R;
        load_full(R, row, tix * C);
        stage(R, tix * C);
        for (int64_t i = 0; i + 1 < left; ++i) {
            const int64_t crow = row, ct0 = tix * C;
            row += dq;
            tix += dr;
            if (tix >= tpr) {
                tix -= tpr;
                ++row;
            }
            load_full(R, row, tix * C);
            compute(crow, ct0, BwdTag<true>{});
            stage(R, tix * C);
            if ((i & (kBwdFlush - 1)) == kBwdFlush - 1) flush();
        }
        compute(row, tix * C, BwdTag<true>{});
    }
    // ragged row ends continue the round-robin order (chunk c to wave c mod nw)
    if (p.n > tpr * C) {
        for (int64_t r = (gw + nw - total % nw) % nw; r < p.rows; r += nw) {
            Regs R;
            load_part(R, r, tpr * C);
            stage(R, tpr * C);
            compute(r, tpr * C, BwdTag<false>{});
        }
    }

    if constexpr (DC) {
        // wave FP64 totals -> block -> one FP32 partial per block, fixed order
        flush();
#pragma unroll
        for (int g = 0; g < NGT; ++g)
            if (64 * g + lane < E) red[wv * E + 64 * g + lane] = tot[g];
        __syncthreads();
        for (int e = tid; e < E; e += kBlock) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) t += red[w * E + e];
            p.partials[(int64_t)blockIdx.x * E + e] = (float)t;
        }
    }
}

template <int NI, int L, bool DX, bool DC>
hipError_t launch_bwd(const BwdParams &p, hipStream_t stream, int grid)
{
    hipLaunchKernelGGL((bwd_kernel<NI, L, DX, DC>), dim3((uint32_t)grid), dim3(kBlock), 0, stream, p);
    return hipGetLastError();
}

template <int NI, int L>
void register_bwd_one(BwdTable &t)
{
    t.fn[NI - 1][L - 1][0] = &launch_bwd<NI, L, true, false>;
    t.fn[NI - 1][L - 1][1] = &launch_bwd<NI, L, false, true>;
    t.fn[NI - 1][L - 1][2] = &launch_bwd<NI, L, true, true>;
    t.kern[NI - 1][L - 1][0] = (const void *)&bwd_kernel<NI, L, true, false>;
    t.kern[NI - 1][L - 1][1] = (const void *)&bwd_kernel<NI, L, false, true>;
    t.kern[NI - 1][L - 1][2] = (const void *)&bwd_kernel<NI, L, true, true>;
}

}  // namespace dpd
