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
// own samples in a fixed order (FP32), the wave and the block reduce in a fixed
// tree, one FP32 partial per block goes to the workspace, and a single block
// sums the partials in FP64 in block order.
#pragma once

#include "dpd_fwd_kernels.h"

namespace dpd {

struct BwdParams {
    const float2 *x;
    const float2 *gz;
    float2 *gx;           // nullptr: no input gradient
    float *partials;      // [gridDim.x][E] (E = 4*L*NI + 2), nullptr: no coeff gradient
    int64_t n, ld, rows;
    int64_t tpr;          // chunks per row (ceil)
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

// Sum over the 64 lanes of a wave (butterfly; every lane gets the total).
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Persistent grid; wave g processes chunks g, g + nw, ... of C = 64*S samples
// (rows flattened, each row zero-padded beyond n).  Per chunk the wave stages
// G (the chunk plus the L-1 samples after it) in a padded wave-private LDS
// buffer; each lane owns S consecutive samples m and reads G_{m..m+S+L-2}.
template <int NI, int L, bool DX, bool DC>
__global__ void __launch_bounds__(kBlock) bwd_kernel(BwdParams p)
{
    constexpr int S = kBwdS;
    constexpr int C = 64 * S;
    constexpr int W = S + L - 1;
    constexpr int NV = S / 2;
    constexpr int WAVES = kBlock / 64;
    constexpr int E = 4 * L * NI + 2;
    constexpr int HS = L - 1;                                   // right halo
    constexpr int SLOTS = 64 * (S + 1) + HS + (HS + S - 1) / S + 1;
    __shared__ __align__(16) float2 gs[WAVES][SLOTS];
    __shared__ float red[DC ? WAVES * E : 1];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const cfloat *M = as_const(p.M);
    float2 *G = gs[wv];
    // slot of chunk-relative sample d (0 <= d < C + HS): one pad after every S
    auto slot = [](int d) { return d + d / S; };

    float acc[DC ? E : 1];
#pragma unroll
    for (int e = 0; e < (DC ? E : 1); ++e) acc[e] = 0.f;

    const int64_t total = p.rows * p.tpr;
    const int64_t nw = (int64_t)gridDim.x * WAVES;
    const int64_t gw = (int64_t)blockIdx.x * WAVES + wv;
    const int hl = HS > 0 ? (lane < HS ? lane : HS - 1) : 0;

    for (int64_t c = gw; c < total; c += nw) {
        const int64_t row = c / p.tpr;
        const int64_t t0 = (c - row * p.tpr) * C;
        const float2 *xr = p.x + row * p.ld;
        const float2 *gr = p.gz + row * p.ld;
        const bool full = t0 + C <= p.n;
        // G chunk (load order: lane l, part i -> samples 2(l + 64 i)) and halo
        float4 gv[NV];
        if (full) {
            const float4 *g4 = reinterpret_cast<const float4 *>(gr + t0);
#pragma unroll
            for (int i = 0; i < NV; ++i) gv[i] = g4[lane + 64 * i];
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int64_t m = t0 + 2 * (lane + 64 * i);
                const float2 u = m < p.n ? gr[m] : make_float2(0.f, 0.f);
                const float2 w = m + 1 < p.n ? gr[m + 1] : make_float2(0.f, 0.f);
                gv[i] = make_float4(u.x, u.y, w.x, w.y);
            }
        }
        float2 gh = make_float2(0.f, 0.f);
        if (HS > 0) {
            const int64_t m = t0 + C + hl;
            const float2 t = gr[m < p.n ? m : p.n - 1];
            gh = m < p.n ? t : make_float2(0.f, 0.f);
        }
        // own samples of x (S consecutive per lane)
        float xa[S], xb[S];
        const int64_t m0 = t0 + (int64_t)lane * S;
        if (full) {
            const float4 *x4 = reinterpret_cast<const float4 *>(xr + m0);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const float4 v = x4[i];
                xa[2 * i] = v.x;
                xb[2 * i] = v.y;
                xa[2 * i + 1] = v.z;
                xb[2 * i + 1] = v.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < S; ++i) {
                const float2 v = m0 + i < p.n ? xr[m0 + i] : make_float2(0.f, 0.f);
                xa[i] = v.x;
                xb[i] = v.y;
            }
        }
        wave_lds_order();
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int j = 2 * (lane + 64 * i);
            G[slot(j)] = make_float2(gv[i].x, gv[i].y);
            G[slot(j) + 1] = make_float2(gv[i].z, gv[i].w);
        }
        if (HS > 0 && lane < HS) G[slot(C + lane)] = gh;
        wave_lds_order();
        float ga[W], gb[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const float2 g = G[slot(lane * S + w)];
            ga[w] = g.x;
            gb[w] = g.y;
        }

        float dxa[S], dxb[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const float a = xa[i], b = xb[i];
            const float s = __builtin_fmaf(a, a, b * b);
            if constexpr (DC) {
                // coefficient gradient: G_{m+k} (x) s^j v
                float pa = a, pb = b;
#pragma unroll
                for (int j = 0; j < NI; ++j) {
#pragma unroll
                    for (int k = 0; k < L; ++k) {
                        float *u = &acc[4 * (k * NI + j)];
                        u[0] = __builtin_fmaf(ga[i + k], pa, u[0]);
                        u[1] = __builtin_fmaf(ga[i + k], pb, u[1]);
                        u[2] = __builtin_fmaf(gb[i + k], pa, u[2]);
                        u[3] = __builtin_fmaf(gb[i + k], pb, u[3]);
                    }
                    pa *= s;
                    pb *= s;
                }
                acc[E - 2] += ga[i];
                acc[E - 1] += gb[i];
            }
            if constexpr (DX) {
                // U_j by taps, then Horner in s for P = sum s^j U_j and
                // Q = sum j s^(j-1) (v . U_j)
                float Pa = 0.f, Pb = 0.f, Q = 0.f;
#pragma unroll
                for (int j = NI - 1; j >= 0; --j) {
                    float ua = 0.f, ub = 0.f;
#pragma unroll
                    for (int k = 0; k < L; ++k) {
                        const cfloat *Mk = M + 4 * (k * NI + j);
                        ua = __builtin_fmaf(Mk[0], ga[i + k], ua);
                        ua = __builtin_fmaf(Mk[2], gb[i + k], ua);
                        ub = __builtin_fmaf(Mk[1], ga[i + k], ub);
                        ub = __builtin_fmaf(Mk[3], gb[i + k], ub);
                    }
                    Pa = __builtin_fmaf(Pa, s, ua);
                    Pb = __builtin_fmaf(Pb, s, ub);
                    if (j > 0) {
                        const float d = __builtin_fmaf(a, ua, b * ub);
                        Q = __builtin_fmaf(Q, s, (float)j * d);
                    }
                }
                const float q2 = 2.f * Q;
                dxa[i] = __builtin_fmaf(q2, a, Pa);
                dxb[i] = __builtin_fmaf(q2, b, Pb);
            }
        }
        if constexpr (DX) {
            float2 *gxr = p.gx + row * p.ld;
            if (full) {
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
#pragma unroll
                for (int i = 0; i < S; ++i)
                    if (m0 + i < p.n) gxr[m0 + i] = make_float2(dxa[i], dxb[i]);
            }
        }
    }

    if constexpr (DC) {
        // wave -> block -> one FP32 partial per block, fixed order
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const float t = wave_sum(acc[e]);
            if (lane == 0) red[wv * E + e] = t;
        }
        __syncthreads();
        for (int e = tid; e < E; e += kBlock) {
            float t = 0.f;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) t += red[w * E + e];
            p.partials[(int64_t)blockIdx.x * E + e] = t;
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
