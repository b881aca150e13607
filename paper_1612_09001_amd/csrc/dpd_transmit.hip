// The forward pass of the coefficient-learning step in one kernel: the
// predistorter (Eq. 1 / Algorithm 1) followed by the two-stage transmitter
// model of the cascade kernels and the loss, so the predistorter output z is
// written once (the adjoint of the cascade reads it) and never read back.
//
// Two forms.  Rows of whole 512-sample chunks on 16-byte aligned buffers take
// the streaming form (transmit_stream_kernel): each wave walks a contiguous
// run of chunks and hands the predistorter outputs that stage B's memory
// needs across lanes and chunks, so each z is computed once.  Other rows take
// the general form: one thread per Q = 8 consecutive samples, which needs
// u = A(z) -- hence z -- at the LB - 1 samples before its own and computes z
// for those too (from the x window reaching L - 1 further back), at
// (Q + LB - 1) / Q of the predistorter's arithmetic.  Everything else --
// the predistorter's filter, stage A, stage B, the loss and dE/dy -- is the
// same arithmetic, in the same order, as dpd_apply_coeffs followed by
// dpd_cascade_loss_grad, so z and dE/dy are bitwise those of the two calls.
// Given device coefficients, every block precombines the predistorter's table
// itself into LDS (no table launch); a table of up to 96 floats then sits in
// VGPRs, a larger one keeps its top Horner level in VGPRs and its lower levels
// in LDS, read tap by tap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>

#include "dpd.h"
#include "dpd_cascade.h"
#include "dpd_fwd_kernels.h"
#include "dpd_plan.h"

#define DPD_EXPORT extern "C" __attribute__((visibility("default")))

namespace dpd {

constexpr int kTxQ = 8;                  // samples per thread
constexpr int kTxNIB = 3, kTxLB = 3;     // stage B this kernel is built for: orders {1,3,5}, 3 taps
constexpr int kTxMaxNI = 5;              // predistorter: orders up to 9
constexpr int kTxMaxL = kSpecL;          // predistorter: up to 8 taps

struct TxParams {
    const float *M;          // predistorter table (used when raw is null)
    const float2 *raw;       // or the K raw coefficients, precombined by every block
    CoefMap map;
    const float *A, *B;      // transmitter stages
    const float2 *x;         // rows x n at stride ld
    float2 *z, *gy;          // outputs, same layout
    int64_t rows, n, ld, qpr;   // qpr = ceil(n / Q) octets per row
    float scale, gscale;
    float *partials;         // one loss partial per block
    int vec;                 // rows start 16-byte aligned: whole octets use 16-byte accesses
};

// Entry e of the predistorter's precombined table (4 L NI matrix floats, then
// c): read from the plan's table, or formed from the raw coefficients with
// the arithmetic of the table kernel (hr+gr, gi-hi, hi+gi, hr-gr), so both give
// the same bits.
__device__ __forceinline__ float tx_table_entry(const TxParams &p, int e)
{
    if (p.raw == nullptr) return p.M[e];
    const int L = p.map.L, NI = p.map.NI;
    if (e >= 4 * L * NI) {
        const float2 c = p.raw[(p.map.n_main + p.map.n_conj) * L];
        return e == 4 * L * NI ? c.x : c.y;
    }
    const int k = e / (4 * NI), r = e - k * 4 * NI, j = r >> 2, q = r & 3;
    float2 h = make_float2(0.f, 0.f), g = make_float2(0.f, 0.f);
    if (p.map.main_idx[j] >= 0) h = p.raw[p.map.main_idx[j] * L + k];
    if (p.map.conj_idx[j] >= 0) g = p.raw[(p.map.n_main + p.map.conj_idx[j]) * L + k];
    return q == 0 ? h.x + g.x : q == 1 ? g.y - h.y : q == 2 ? h.y + g.y : h.x - g.x;
}

// The predistorter's filter for tables too large for registers: the top
// Horner level of every tap in VGPRs (`top`), the lower levels of each tap
// read from the LDS copy of the table just before the tap is used, the
// arithmetic in the order of fir_outputs (the same bits).
template <int NI, int L, int S>
__device__ __forceinline__ void tx_fir_lds(const float (&a)[S + L - 1], const float (&b)[S + L - 1],
                                           const float (&s)[S + L - 1], const float (&top)[4 * L],
                                           const float *CS, float (&zr)[S], float (&zi)[S])
{
    constexpr int T = 4 * (NI - 1);
    // An opaque zero keeps the table reads inside the caller's chunk loop:
    // hoisted, every tap's lower levels would hold registers for the whole
    // kernel.
    int zo = 0;
    asm volatile("" : "+v"(zo));
    CS += zo;
    const float2 c0 = *reinterpret_cast<const float2 *>(CS + 4 * L * NI);
#pragma unroll
    for (int i = 0; i < S; ++i) {
        zr[i] = c0.x;
        zi[i] = c0.y;
    }
#pragma unroll
    for (int k = 0; k < L; ++k) {
        float c[T > 0 ? T : 1];
        const float4 *ck = reinterpret_cast<const float4 *>(CS + 4 * NI * k);
#pragma unroll
        for (int j = 0; j < NI - 1; ++j) {
            const float4 u = ck[j];
            c[4 * j + 0] = u.x;
            c[4 * j + 1] = u.y;
            c[4 * j + 2] = u.z;
            c[4 * j + 3] = u.w;
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const int w = i + (L - 1) - k;
            float w00 = top[4 * k + 0], w01 = top[4 * k + 1];
            float w10 = top[4 * k + 2], w11 = top[4 * k + 3];
#pragma unroll
            for (int j = NI - 2; j >= 0; --j) {
                w00 = __builtin_fmaf(w00, s[w], c[4 * j + 0]);
                w01 = __builtin_fmaf(w01, s[w], c[4 * j + 1]);
                w10 = __builtin_fmaf(w10, s[w], c[4 * j + 2]);
                w11 = __builtin_fmaf(w11, s[w], c[4 * j + 3]);
            }
            zr[i] = __builtin_fmaf(w00, a[w], zr[i]);
            zr[i] = __builtin_fmaf(w01, b[w], zr[i]);
            zi[i] = __builtin_fmaf(w10, a[w], zi[i]);
            zi[i] = __builtin_fmaf(w11, b[w], zi[i]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int NI, int L>
__global__ void __launch_bounds__(kBlock) transmit_fwd_kernel(TxParams p)
{
    constexpr int NIB = kTxNIB, LB = kTxLB, Q = kTxQ;
    constexpr int ZW = Q + LB - 1;           // z and u at m0 - (LB - 1) .. m0 + Q - 1
    constexpr int XW = ZW + L - 1;           // x at m0 - (LB - 1) - (L - 1) .. m0 + Q - 1
    constexpr int XH = XW - Q;               // x samples before m0
    constexpr int NC = 4 * L * NI + 2;
    constexpr bool REG = NC <= kRegCoefMax;
    constexpr int NB = 4 * LB * NIB + 2;     // stage-B table floats
    __shared__ double red[kBlock];
    __shared__ __align__(16) float mtab[NC + 2];
    __shared__ float tab[NB + 6];

    // The predistorter's table into LDS (small tables then into VGPRs; larger
    // ones are read tap by tap from LDS), the stage tables through LDS into
    // VGPRs.  Stage A is memoryless with one power level: u = c + M0 z.
    const int tid = threadIdx.x;
    if (tid < NC)
        mtab[tid] = tx_table_entry(p, tid);
    else if (tid < NC + NB)
        tab[tid - NC] = p.B[tid - NC];
    else if (tid < NC + NB + 6)
        tab[tid - NC] = p.A[tid - NC - NB];
    __syncthreads();
    float coef[REG ? NC : 1], top[REG ? 1 : 4 * L];
    if constexpr (REG) {
#pragma unroll
        for (int e = 0; e < NC; ++e) coef[e] = mtab[e];
    } else {
#pragma unroll
        for (int k = 0; k < L; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) top[4 * k + q] = mtab[4 * NI * k + 4 * (NI - 1) + q];
    }
    float tb[NB], ta[6];
#pragma unroll
    for (int e = 0; e < NB; ++e) tb[e] = tab[e];
#pragma unroll
    for (int e = 0; e < 6; ++e) ta[e] = tab[NB + e];

    LossSum ls;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t q0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    CasWalk wk(q0, stride, p.qpr);
    for (; wk.row < p.rows; wk.next(p.qpr)) {
        const int64_t m0 = wk.k * Q;
        const float2 *xr = p.x + wk.row * p.ld;
        float2 *zrow = p.z + wk.row * p.ld;
        float2 *grow = p.gy + wk.row * p.ld;
        const bool vec = p.vec && m0 + Q <= p.n;
        float a[XW], b[XW], s[XW];
        if (vec) {
            const float4 *x4 = reinterpret_cast<const float4 *>(xr + m0);
#pragma unroll
            for (int i = 0; i < Q / 2; ++i) {
                const float4 v = x4[i];
                a[XH + 2 * i] = v.x;
                b[XH + 2 * i] = v.y;
                a[XH + 2 * i + 1] = v.z;
                b[XH + 2 * i + 1] = v.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const float2 v = cas_load(xr, m0 + i, p.n);
                a[XH + i] = v.x;
                b[XH + i] = v.y;
            }
        }
#pragma unroll
        for (int w = 0; w < XH; ++w) {
            const float2 v = cas_load(xr, m0 - XH + w, p.n);   // zero before the row start
            a[w] = v.x;
            b[w] = v.y;
        }
#pragma unroll
        for (int w = 0; w < XW; ++w) s[w] = __builtin_fmaf(a[w], a[w], b[w] * b[w]);
        // the predistorter at the ZW samples ending with this thread's last
        float zr[ZW], zi[ZW];
        if constexpr (REG)
            fir_outputs_reg<NI, L, ZW>(a, b, s, coef, zr, zi);
        else
            tx_fir_lds<NI, L, ZW>(a, b, s, top, mtab, zr, zi);
        // u = A(z); zero before the row start (stage B's zero history)
        float2 u[ZW];
        float su[ZW];
#pragma unroll
        for (int w = 0; w < ZW; ++w) {
            const int64_t m = m0 - (LB - 1) + w;
            // A(z) = c + M0 z, the arithmetic of the cascade kernels' stage A at one level
            const float ur = __builtin_fmaf(ta[0], zr[w], __builtin_fmaf(ta[1], zi[w], ta[4]));
            const float ui = __builtin_fmaf(ta[2], zr[w], __builtin_fmaf(ta[3], zi[w], ta[5]));
            u[w] = (m >= 0 && m < p.n) ? make_float2(ur, ui) : make_float2(0.f, 0.f);
            su[w] = __builtin_fmaf(u[w].x, u[w].x, u[w].y * u[w].y);
        }
        float2 g[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            float yr = tb[4 * LB * NIB], yi = tb[4 * LB * NIB + 1];
#pragma unroll
            for (int k = 0; k < LB; ++k) {
                const int w = i + (LB - 1) - k;
                const float *t = tb + 4 * NIB * k;
                float w00 = t[4 * (NIB - 1)], w01 = t[4 * (NIB - 1) + 1];
                float w10 = t[4 * (NIB - 1) + 2], w11 = t[4 * (NIB - 1) + 3];
#pragma unroll
                for (int j = NIB - 2; j >= 0; --j) {
                    w00 = __builtin_fmaf(w00, su[w], t[4 * j + 0]);
                    w01 = __builtin_fmaf(w01, su[w], t[4 * j + 1]);
                    w10 = __builtin_fmaf(w10, su[w], t[4 * j + 2]);
                    w11 = __builtin_fmaf(w11, su[w], t[4 * j + 3]);
                }
                yr = __builtin_fmaf(w00, u[w].x, __builtin_fmaf(w01, u[w].y, yr));
                yi = __builtin_fmaf(w10, u[w].x, __builtin_fmaf(w11, u[w].y, yi));
            }
            const bool in = m0 + i < p.n;
            const float rr = in ? __builtin_fmaf(p.scale, yr, -a[XH + i]) : 0.f;
            const float ri = in ? __builtin_fmaf(p.scale, yi, -b[XH + i]) : 0.f;
            ls.f = __builtin_fmaf(rr, rr, __builtin_fmaf(ri, ri, ls.f));
            g[i] = make_float2(p.gscale * rr, p.gscale * ri);
        }
        if (vec) {
            float4 *z4 = reinterpret_cast<float4 *>(zrow + m0);
            float4 *g4 = reinterpret_cast<float4 *>(grow + m0);
#pragma unroll
            for (int i = 0; i < Q / 2; ++i) {
                z4[i] = make_float4(zr[LB - 1 + 2 * i], zi[LB - 1 + 2 * i], zr[LB + 2 * i], zi[LB + 2 * i]);
                g4[i] = make_float4(g[2 * i].x, g[2 * i].y, g[2 * i + 1].x, g[2 * i + 1].y);
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i)
                if (m0 + i < p.n) {
                    zrow[m0 + i] = make_float2(zr[LB - 1 + i], zi[LB - 1 + i]);
                    grow[m0 + i] = g[i];
                }
        }
        ls.step_done();
    }
    red[threadIdx.x] = ls.total();
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) p.partials[blockIdx.x] = (float)red[0];
}

// lane l receives v of lane l - 1; lane 0 receives `first` (wave-uniform)
__device__ __forceinline__ float shift_up(float v, float first)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(first), __float_as_int(v), 0x138, 0xf, 0xf, false));
}

// The same pass for rows made of whole 512-sample chunks, on the streaming
// forward kernel's machinery: persistent waves, each taking a contiguous run
// of chunks (wave g: chunks g * per .. (g + 1) * per - 1 of the flattened
// rows), every chunk register-prefetched one ahead with coalesced 16-byte
// loads and staged through wave-private LDS for the predistorter's windows.
// Lane l filters samples 8l .. 8l + 7 of a chunk; the two predistorter outputs
// before them, which stage B's memory needs, come from lane l - 1 by a DPP
// shift, and for lane 0 from the previous chunk of the run (its lane 63),
// or -- at the start of a run inside a row -- from a direct evaluation by
// lanes 0 and 1.  z and dE/dy leave through LDS as 1 KiB stores.
template <int NI, int L>
__global__ void __launch_bounds__(kBlock) transmit_stream_kernel(TxParams p)
{
    constexpr int NIB = kTxNIB, LB = kTxLB;
    static_assert(LB == 3, "the shifted halo holds two outputs");
    constexpr int S = 8, C = 64 * S, W = S + L - 1, NV = S / 2, WAVES = kBlock / 64;
    using PL = PadLayout<L, S>;
    constexpr int HS = L - 1;
    constexpr int NC = 4 * L * NI + 2;
    constexpr bool REG = NC <= kRegCoefMax;
    constexpr int NB = 4 * LB * NIB + 2;
    __shared__ __align__(16) float mtab[NC + 2];
    __shared__ float tab[REG ? NB + 6 : 1];
    __shared__ __align__(16) float2 xs[WAVES][PL::SLOTS];
    __shared__ __align__(16) float ss[WAVES][PL::SLOTS];
    __shared__ double red[WAVES];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (tid < NC)
        mtab[tid] = tx_table_entry(p, tid);
    else if (REG && tid < NC + NB)
        tab[tid - NC] = p.B[tid - NC];
    else if (REG && tid < NC + NB + 6)
        tab[tid - NC] = p.A[tid - NC - NB];
    __syncthreads();
    float coef[REG ? NC : 1], top[REG ? 1 : 4 * L];
    if constexpr (REG) {
#pragma unroll
        for (int e = 0; e < NC; ++e) coef[e] = mtab[e];
    } else {
#pragma unroll
        for (int k = 0; k < L; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) top[4 * k + q] = mtab[4 * NI * k + 4 * (NI - 1) + q];
    }
    // the stage tables: per-lane copies through LDS beside a register-resident
    // predistorter table; wave-uniform (scalar) operands beside an LDS-resident
    // one, whose lower levels leave the scalar registers free
    float tb[NB], ta[6];
#pragma unroll
    for (int e = 0; e < NB; ++e) tb[e] = REG ? tab[e] : p.B[e];
#pragma unroll
    for (int e = 0; e < 6; ++e) ta[e] = REG ? tab[NB + e] : p.A[e];

    float2 *X = xs[wv];
    float *SX = ss[wv];
    const int64_t tpr = p.n / C;
    const int64_t total = p.rows * tpr;
    const int64_t nw = (int64_t)gridDim.x * WAVES;
    const int64_t gw = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * WAVES + wv;
    const int64_t per = (total + nw - 1) / nw;
    const int64_t c_begin = gw * per < total ? gw * per : total;
    const int64_t c_end = c_begin + per < total ? c_begin + per : total;
    const int hl = HS > 0 ? (lane < HS ? lane : HS - 1) : 0;
    LossSum ls;   // this lane's share, flushed to FP64 every kLossFlush chunks

    struct Cur {
        int64_t row, k;
    };
    // raw halo sample (hl - HS) of a chunk: read from the row start at t0 < HS
    auto halo_raw = [&](const Cur &u) {
        const int64_t t0 = u.k * C;
        const int64_t off = t0 >= HS ? t0 - HS : 0;
        const cfloat *hp = as_const(reinterpret_cast<const float *>(p.x + u.row * p.ld + off));
        float2 r = make_float2(hp[0], hp[1]);
#pragma unroll
        for (int k = 1; k < (HS > 0 ? HS : 1); ++k)
            if (hl == k) r = make_float2(hp[2 * k], hp[2 * k + 1]);
        return r;
    };
    auto load_full = [&](ChunkRegs<S> &buf, const Cur &u) {
        __builtin_amdgcn_s_setprio(2);   // the prefetch at raised wave priority
        const float4 *x4 = reinterpret_cast<const float4 *>(p.x + u.row * p.ld + u.k * C);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const v4f t = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(x4) + lane + 64 * i);
            buf.v[i] = make_float4(t.x, t.y, t.z, t.w);
        }
        buf.h = halo_raw(u);
        __builtin_amdgcn_s_setprio(0);
    };
    auto next = [&](Cur u) {
        if (++u.k == tpr) {
            u.k = 0;
            ++u.row;
        }
        return u;
    };

    // the predistorter outputs before a run's first chunk (mid-row): lanes 0
    // and 1 evaluate samples t0 - 2 and t0 - 1 directly (same arithmetic)
    float cz[4] = {0.f, 0.f, 0.f, 0.f};   // z_r, z_i at t0 - 2, then at t0 - 1 (wave-uniform)
    if (c_begin < c_end) {
        const int64_t row = c_begin / tpr, t0 = (c_begin - row * tpr) * C;
        if (t0 > 0) {
            const int64_t m = t0 - 2 + (lane & 1);
            const float2 *xr = p.x + row * p.ld;
            float a[L], b[L], sv[L];
#pragma unroll
            for (int w = 0; w < L; ++w) {
                const float2 v = xr[m - (L - 1) + w];
                a[w] = v.x;
                b[w] = v.y;
                sv[w] = __builtin_fmaf(v.x, v.x, v.y * v.y);
            }
            float zr1[1], zi1[1];
            if constexpr (REG)
                fir_outputs_reg<NI, L, 1>(a, b, sv, coef, zr1, zi1);
            else
                tx_fir_lds<NI, L, 1>(a, b, sv, top, mtab, zr1, zi1);
            cz[0] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zr1[0]), 0));
            cz[1] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zi1[0]), 0));
            cz[2] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zr1[0]), 1));
            cz[3] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zi1[0]), 1));
        }
    }

    auto step = [&](const ChunkRegs<S> &buf, const Cur &u) {
        const int64_t t0 = u.k * C;
        // samples and |x|^2 into LDS
        wave_lds_order();
        if (HS > 0 && lane < HS) {
            float2 h = buf.h;
            if (t0 - HS + lane < 0) h = make_float2(0.f, 0.f);
            const int q = PL::slot(lane - HS);
            X[q] = h;
            SX[q] = __builtin_fmaf(h.x, h.x, h.y * h.y);
        }
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const float4 v = buf.v[i];
            const int j = 2 * (lane + 64 * i);
            const int q = PL::OFF + j + j / S;
            X[q] = make_float2(v.x, v.y);
            X[q + 1] = make_float2(v.z, v.w);
            SX[q] = __builtin_fmaf(v.x, v.x, v.y * v.y);
            SX[q + 1] = __builtin_fmaf(v.z, v.z, v.w * v.w);
        }
        wave_lds_order();
        float a[W], b[W], sw[W];
        const int lb = lane * (S + 1);
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int q = lb + PL::slot(w - (L - 1));
            const float2 v = X[q];
            a[w] = v.x;
            b[w] = v.y;
            sw[w] = SX[q];
        }
        float zr[S], zi[S];
        if constexpr (REG)
            fir_outputs_reg<NI, L, S>(a, b, sw, coef, zr, zi);
        else
            tx_fir_lds<NI, L, S>(a, b, sw, top, mtab, zr, zi);
        // z at the two samples before this lane's: lane l - 1, or the carry
        float zh[4];
        zh[0] = shift_up(zr[S - 2], cz[0]);
        zh[1] = shift_up(zi[S - 2], cz[1]);
        zh[2] = shift_up(zr[S - 1], cz[2]);
        zh[3] = shift_up(zi[S - 1], cz[3]);
        cz[0] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zr[S - 2]), 63));
        cz[1] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zi[S - 2]), 63));
        cz[2] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zr[S - 1]), 63));
        cz[3] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zi[S - 1]), 63));
        // u = A(z) on samples 8l - 2 .. 8l + 7; zero before the row start
        constexpr int ZW = S + LB - 1;
        float2 uu[ZW];
        float su[ZW];
#pragma unroll
        for (int w = 0; w < ZW; ++w) {
            const float r = w < LB - 1 ? zh[2 * w] : zr[w - (LB - 1)];
            const float i = w < LB - 1 ? zh[2 * w + 1] : zi[w - (LB - 1)];
            const float ur = __builtin_fmaf(ta[0], r, __builtin_fmaf(ta[1], i, ta[4]));
            const float ui = __builtin_fmaf(ta[2], r, __builtin_fmaf(ta[3], i, ta[5]));
            const bool before = t0 == 0 && lane == 0 && w < LB - 1;
            uu[w] = before ? make_float2(0.f, 0.f) : make_float2(ur, ui);
            su[w] = __builtin_fmaf(uu[w].x, uu[w].x, uu[w].y * uu[w].y);
        }
        float gr[S], gi[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            float yr = tb[4 * LB * NIB], yi = tb[4 * LB * NIB + 1];
#pragma unroll
            for (int k = 0; k < LB; ++k) {
                const int w = i + (LB - 1) - k;
                const float *t = tb + 4 * NIB * k;
                float w00 = t[4 * (NIB - 1)], w01 = t[4 * (NIB - 1) + 1];
                float w10 = t[4 * (NIB - 1) + 2], w11 = t[4 * (NIB - 1) + 3];
#pragma unroll
                for (int j = NIB - 2; j >= 0; --j) {
                    w00 = __builtin_fmaf(w00, su[w], t[4 * j + 0]);
                    w01 = __builtin_fmaf(w01, su[w], t[4 * j + 1]);
                    w10 = __builtin_fmaf(w10, su[w], t[4 * j + 2]);
                    w11 = __builtin_fmaf(w11, su[w], t[4 * j + 3]);
                }
                yr = __builtin_fmaf(w00, uu[w].x, __builtin_fmaf(w01, uu[w].y, yr));
                yi = __builtin_fmaf(w10, uu[w].x, __builtin_fmaf(w11, uu[w].y, yi));
            }
            const float rr = __builtin_fmaf(p.scale, yr, -a[L - 1 + i]);
            const float ri = __builtin_fmaf(p.scale, yi, -b[L - 1 + i]);
            ls.f = __builtin_fmaf(rr, rr, __builtin_fmaf(ri, ri, ls.f));
            gr[i] = p.gscale * rr;
            gi[i] = p.gscale * ri;
        }
        // z, then dE/dy, back through LDS: every store writes 1 KiB
        float2 *zrow = p.z + u.row * p.ld + t0;
        float2 *grow = p.gy + u.row * p.ld + t0;
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            wave_lds_order();
            const int ob = lane * (S + 1) + PL::OFF;
#pragma unroll
            for (int i = 0; i < S; ++i)
                X[ob + i] = pass == 0 ? make_float2(zr[i], zi[i]) : make_float2(gr[i], gi[i]);
            wave_lds_order();
            v4f *o4 = reinterpret_cast<v4f *>(pass == 0 ? zrow : grow);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int j = 2 * (lane + 64 * i);
                const int q = PL::OFF + j + j / S;
                const float2 u0 = X[q], u1 = X[q + 1];
                const v4f v = {u0.x, u0.y, u1.x, u1.y};
                __builtin_nontemporal_store(v, o4 + lane + 64 * i);
            }
        }
        ls.step_done();
    };

    if (c_begin < c_end) {
        int64_t left = c_end - c_begin;
        Cur cur;
        cur.row = c_begin / tpr;
        cur.k = c_begin - cur.row * tpr;
        ChunkRegs<S> A, B;
        load_full(A, cur);
        for (; left >= 3; left -= 2) {
            const Cur c1 = next(cur);
            load_full(B, c1);
            step(A, cur);
            const Cur c2 = next(c1);
            load_full(A, c2);
            step(B, c1);
            cur = c2;
        }
        if (left == 2) {
            const Cur c1 = next(cur);
            load_full(B, c1);
            step(A, cur);
            step(B, c1);
        } else {
            step(A, cur);
        }
    }
    // wave -> block -> one loss partial per block (fixed order, FP64)
    double acc = ls.total();
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = red[0];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) t += red[w];
        p.partials[blockIdx.x] = (float)t;
    }
}

typedef void (*TxKernel)(TxParams);

template <int NI, int L>
struct TxEntry {
    static void fill(TxKernel (&f)[kTxMaxNI][kTxMaxL], TxKernel (&g)[kTxMaxNI][kTxMaxL])
    {
        f[NI - 1][L - 1] = &transmit_fwd_kernel<NI, L>;
        g[NI - 1][L - 1] = &transmit_stream_kernel<NI, L>;
        if constexpr (L < kTxMaxL)
            TxEntry<NI, L + 1>::fill(f, g);
        else if constexpr (NI < kTxMaxNI)
            TxEntry<NI + 1, 1>::fill(f, g);
    }
};

struct TxTable {
    TxKernel fwd[kTxMaxNI][kTxMaxL];
    TxKernel stream[kTxMaxNI][kTxMaxL];
    TxTable() { TxEntry<1, 1>::fill(fwd, stream); }
};

static const TxTable &tx_table()
{
    static const TxTable t;
    return t;
}

int num_cus();

// Resident blocks per CU of one instance (queried once per instance).
static int tx_occupancy(int NI, int L, int which, const void *kern)
{
    static std::atomic<int> cache[2][kTxMaxNI][kTxMaxL] = {};
    int v = cache[which][NI - 1][L - 1].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kern, kBlock, 0) != hipSuccess || v < 1) v = 1;
        cache[which][NI - 1][L - 1].store(v, std::memory_order_relaxed);
    }
    return v;
}

hipError_t launch_transmit_forward(const dpd_plan *P, const dpd_plan *A, const dpd_plan *B, hipStream_t hs,
                                   const void *coeffs_dev, const void *x, void *z, void *grad_y, int64_t rows,
                                   int64_t n, int64_t ld, float scale, float *partials, int *nblk)
{
    *nblk = 0;
    const int64_t N = rows * n;
    if (N == 0) return hipSuccess;
    TxParams p;
    p.M = P->d_table;
    p.raw = (const float2 *)coeffs_dev;
    p.map = P->map;
    p.A = A->d_table;
    p.B = B->d_table;
    p.x = (const float2 *)x;
    p.z = (float2 *)z;
    p.gy = (float2 *)grad_y;
    p.rows = rows;
    p.n = n;
    p.ld = rows > 1 ? ld : n;
    p.qpr = (n + kTxQ - 1) / kTxQ;
    p.scale = scale;
    p.gscale = (float)(2.0 * scale / (double)N);
    p.partials = partials;
    p.vec = ((uintptr_t)x % 16 == 0 && (uintptr_t)z % 16 == 0 && (uintptr_t)grad_y % 16 == 0 &&
             (rows == 1 || ld % 2 == 0)) ? 1 : 0;
    // whole 512-sample chunks on 16-byte aligned rows: the streaming form,
    // at most two resident blocks per CU; else one thread per eight
    // samples.  One round of resident blocks either way (a second partial
    // round would double the tail).
    const bool stream_form = p.vec && n % 512 == 0;
    const TxKernel kern = (stream_form ? tx_table().stream : tx_table().fwd)[P->map.NI - 1][P->map.L - 1];
    const int occ = tx_occupancy(P->map.NI, P->map.L, stream_form ? 1 : 0, (const void *)kern);
    const int64_t cap = (int64_t)num_cus() * (stream_form ? std::min(occ, 2) : occ);
    const int64_t work = stream_form ? (rows * (n / 512) + 3) / 4 : (rows * p.qpr + kBlock - 1) / kBlock;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(kLossBlocks, cap), work));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, hs, p);
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) *nblk = grid;
    return e;
}

}  // namespace dpd

using namespace dpd;

namespace dpd {

dpd_status check_transmit_forward(const dpd_plan *P, const dpd_plan *A, const dpd_plan *B, const void *x,
                                  const void *z, const void *grad_y, int64_t rows, int64_t n, int64_t ld,
                                  float scale)
{
    if (P == nullptr || A == nullptr || B == nullptr) return DPD_EINVAL;
    if (A->map.L != 1) return DPD_EINVAL;
    if (rows < 0 || n < 0 || (rows > 1 && ld < n)) return DPD_EINVAL;
    if (!std::isfinite(scale)) return DPD_EINVAL;
    if (A->map.NI != 1 || B->map.NI != kTxNIB || B->map.L != kTxLB || P->map.NI > kTxMaxNI ||
        P->map.L > kTxMaxL)
        return DPD_EUNSUPPORTED;
    if (rows * n > 0) {
        if (x == nullptr || z == nullptr || grad_y == nullptr) return DPD_EINVAL;
        for (const void *q : {x, z, grad_y})
            if ((uintptr_t)q % 8 != 0) return DPD_EINVAL;
        const size_t span = (size_t)(((rows - 1) * (rows > 1 ? ld : n) + n) * (int64_t)sizeof(float2));
        const auto lap = [&](const void *a, const void *b) {
            const uintptr_t u = (uintptr_t)a, v = (uintptr_t)b;
            return u < v + span && v < u + span;
        };
        if (lap(z, x) || lap(grad_y, x) || lap(z, grad_y)) return DPD_EINVAL;
    }
    return DPD_OK;
}

}  // namespace dpd

DPD_EXPORT dpd_status dpd_transmit_loss_grad(dpd_plan *P, const dpd_plan *A, const dpd_plan *B, void *stream,
                                             const void *coeffs_dev, const void *x, void *z, int64_t rows, int64_t n,
                                             int64_t ld, float scale, float *loss_dev, void *grad_y, void *ws,
                                             size_t ws_bytes)
{
    const dpd_status st = check_transmit_forward(P, A, B, x, z, grad_y, rows, n, ld, scale);
    if (st != DPD_OK) return st;
    if (ws == nullptr || ws_bytes < kLossBlocks * sizeof(float) || (uintptr_t)ws % 4 != 0) return DPD_EINVAL;
    if (coeffs_dev != nullptr && (uintptr_t)coeffs_dev % 8 != 0) return DPD_EINVAL;
    const int64_t N = rows * n;
    const hipStream_t hs = (hipStream_t)stream;
    int nblk = 0;
    hipError_t e =
        launch_transmit_forward(P, A, B, hs, coeffs_dev, x, z, grad_y, rows, n, ld, scale, (float *)ws, &nblk);
    if (e != hipSuccess) return hip_fail(e);
    if (loss_dev != nullptr) {
        e = launch_loss_finalize((const float *)ws, nblk, N > 0 ? 1.0 / (double)N : 0.0, loss_dev, hs);
        if (e != hipSuccess) return hip_fail(e);
    }
    return DPD_OK;
}
