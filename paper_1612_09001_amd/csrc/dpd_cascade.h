// Pieces of the transmitter-cascade kernels shared by the training
// translation units (dpd_train.hip, dpd_transmit.hip, dpd_transmit_bwd.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "dpd_internal.h"
#include "dpd_plan.h"
#include "dpd_reduce.h"

namespace dpd {

constexpr int kLossBlocks = 1024;   // loss partials (one per block of the loss kernels)

// A thread's (or lane's) share of a loss sum: FP32 over at most kLossFlush
// loop steps, then added to an FP64 total, so the rounding error does not grow
// with the number of samples one thread sums.
constexpr int kLossFlush = 32;
struct LossSum {
    float f = 0.f;
    double d = 0.0;
    int c = 0;
    __device__ __forceinline__ void step_done()
    {
        if (++c == kLossFlush) {
            d += (double)f;
            f = 0.f;
            c = 0;
        }
    }
    __device__ __forceinline__ double total() const { return d + (double)f; }
};

constexpr int kCasTA = 4 * kMaxNI + 2;   // stage-A table floats held in registers (at most)

// A(z) for one sample (memoryless: c + W(|z|^2) z, W by Horner over NIA
// levels from the top one down)
__device__ __forceinline__ float2 cas_stage_a(const float (&T)[kCasTA], int NIA, float2 v)
{
    float w00 = T[0], w01 = T[1], w10 = T[2], w11 = T[3];
    if (NIA > 1) {
        const float s = __builtin_fmaf(v.x, v.x, v.y * v.y);
#pragma unroll
        for (int j = kMaxNI - 1; j >= 0; --j) {
            if (j == NIA - 1) {
                w00 = T[4 * j + 0];
                w01 = T[4 * j + 1];
                w10 = T[4 * j + 2];
                w11 = T[4 * j + 3];
            } else if (j < NIA - 1) {
                w00 = __builtin_fmaf(w00, s, T[4 * j + 0]);
                w01 = __builtin_fmaf(w01, s, T[4 * j + 1]);
                w10 = __builtin_fmaf(w10, s, T[4 * j + 2]);
                w11 = __builtin_fmaf(w11, s, T[4 * j + 3]);
            }
        }
    }
    float cr = T[4 * kMaxNI], ci = T[4 * kMaxNI + 1];
#pragma unroll
    for (int j = kMaxNI - 1; j >= 1; --j)
        if (j == NIA) {
            cr = T[4 * j];
            ci = T[4 * j + 1];
        }
    return make_float2(__builtin_fmaf(w00, v.x, __builtin_fmaf(w01, v.y, cr)),
                       __builtin_fmaf(w10, v.x, __builtin_fmaf(w11, v.y, ci)));
}

// P + 2 Q v of the adjoint of a map at v from its U_j (levels j < NI):
// P = sum_j s^j U_j and Q = sum_j j s^(j-1) v.U_j by Horner, s = |v|^2.
template <int NI>
__device__ __forceinline__ float2 cas_adjoint_sum(const float (&Ux)[NI], const float (&Uy)[NI], float2 v)
{
    if constexpr (NI == 1) {
        return make_float2(Ux[0], Uy[0]);
    } else {
        const float s = __builtin_fmaf(v.x, v.x, v.y * v.y);
        float px = Ux[NI - 1], py = Uy[NI - 1];
        float q = (float)(NI - 1) * __builtin_fmaf(v.x, Ux[NI - 1], v.y * Uy[NI - 1]);
        px = __builtin_fmaf(px, s, Ux[NI - 2]);
        py = __builtin_fmaf(py, s, Uy[NI - 2]);
#pragma unroll
        for (int j = NI - 2; j >= 1; --j) {
            q = __builtin_fmaf(q, s, (float)j * __builtin_fmaf(v.x, Ux[j], v.y * Uy[j]));
            px = __builtin_fmaf(px, s, Ux[j - 1]);
            py = __builtin_fmaf(py, s, Uy[j - 1]);
        }
        return make_float2(__builtin_fmaf(2.f * q, v.x, px), __builtin_fmaf(2.f * q, v.y, py));
    }
}

// Adjoint of stage B (NIB levels, LB taps, table tb) at u_m = uv:
// U_j = sum_k M_{j,k}^T g_{m+k} from g[0..LB-1] = dE/dy at m .. m + LB - 1.
template <int NIB, int LB>
__device__ __forceinline__ float2 cas_b_adjoint(const float *tb, const float2 *g, float2 uv)
{
    float Ux[NIB], Uy[NIB];
#pragma unroll
    for (int j = 0; j < NIB; ++j) {
        float ax = 0.f, ay = 0.f;
#pragma unroll
        for (int k = 0; k < LB; ++k) {
            const float *t = tb + 4 * (k * NIB + j);
            ax = __builtin_fmaf(t[0], g[k].x, __builtin_fmaf(t[2], g[k].y, ax));
            ay = __builtin_fmaf(t[1], g[k].x, __builtin_fmaf(t[3], g[k].y, ay));
        }
        Ux[j] = ax;
        Uy[j] = ay;
    }
    return cas_adjoint_sum<NIB>(Ux, Uy, uv);
}

// Adjoint of the memoryless stage A (one tap, NIA levels) at z from gu:
// V_j = M_j^T gu, then P + 2 Q z by Horner from the top level down (one level:
// the transpose alone).
__device__ __forceinline__ float2 cas_a_adjoint(const float (&ta)[kCasTA], int NIA, float2 z1, float2 gu)
{
    const float v0x = __builtin_fmaf(ta[0], gu.x, ta[2] * gu.y);
    const float v0y = __builtin_fmaf(ta[1], gu.x, ta[3] * gu.y);
    if (NIA == 1) return make_float2(v0x, v0y);
    const float sa = __builtin_fmaf(z1.x, z1.x, z1.y * z1.y);
    float px = 0.f, py = 0.f, qa = 0.f;
#pragma unroll
    for (int j = kMaxNI - 1; j >= 1; --j) {
        if (j < NIA) {
            const float vx = __builtin_fmaf(ta[4 * j + 0], gu.x, ta[4 * j + 2] * gu.y);
            const float vy = __builtin_fmaf(ta[4 * j + 1], gu.x, ta[4 * j + 3] * gu.y);
            const float d = (float)j * __builtin_fmaf(z1.x, vx, z1.y * vy);
            if (j == NIA - 1) {
                px = vx;
                py = vy;
                qa = d;
            } else {
                px = __builtin_fmaf(px, sa, vx);
                py = __builtin_fmaf(py, sa, vy);
                qa = __builtin_fmaf(qa, sa, d);
            }
        }
    }
    px = __builtin_fmaf(px, sa, v0x);
    py = __builtin_fmaf(py, sa, v0y);
    return make_float2(__builtin_fmaf(2.f * qa, z1.x, px), __builtin_fmaf(2.f * qa, z1.y, py));
}

// FP64 total of nblk FP32 loss partials by one block of kBlock threads: each
// thread its strided share in order, the DPP lane sum of each wave, then the
// waves in order; the result is valid in thread 0.
__device__ __forceinline__ double loss_block_total(const float *__restrict__ partials, int nblk,
                                                   double (&red)[kBlock / 64])
{
    double t = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) t += (double)partials[b];
    t = wave_sum_to_lane63(t);
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = t;
    __syncthreads();
    double u = red[0];
    for (int w = 1; w < kBlock / 64; ++w) u += red[w];
    return u;
}

// One Adam update (Kingma & Ba) of a real parameter from its gradient g;
// bc1, bc2 are the bias corrections 1 - beta^step.
__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, float lr, float b1, float b2,
                                         float eps, float bc1, float bc2)
{
    const float mi = __builtin_fmaf(b1, m, (1.f - b1) * g);
    const float vi = __builtin_fmaf(b2, v, (1.f - b2) * g * g);
    m = mi;
    v = vi;
    const float denom = __builtin_sqrtf(vi / bc2) + eps;
    p -= (lr / bc1) * mi / denom;
}

__device__ __forceinline__ float2 cas_load(const float2 *__restrict__ r, int64_t m, int64_t n)
{
    return (m >= 0 && m < n) ? r[m] : make_float2(0.f, 0.f);
}

// This thread's quads: (row, quad) starting at q0 and advanced by the grid
// stride without a division.
struct CasWalk {
    int64_t row, k, dr, dk;
    __device__ CasWalk(int64_t q0, int64_t stride, int64_t qpr)
        : row(q0 / qpr), k(q0 - (q0 / qpr) * qpr), dr(stride / qpr), dk(stride - (stride / qpr) * qpr) {}
    __device__ void next(int64_t qpr)
    {
        row += dr;
        k += dk;
        if (k >= qpr) {
            k -= qpr;
            ++row;
        }
    }
};

// FP64 sum of loss partials into *loss (one block; dpd_train.hip).
hipError_t launch_loss_finalize(const float *partials, int nblk, double inv_n, float *loss, hipStream_t st);

// Coefficient-gradient partials of the predistorter's backward (dpd_bwd.hip):
// the workspace bytes one call needs, and the FP64 finalisation of nblk
// per-block partials into K complex gradients.
size_t bwd_ws_bytes(const CoefMap &map);

// Argument checks of the one-pass forward of the learning step (the stages
// it is built for, sizes, alignment, overlaps; not the workspace).
dpd_status check_transmit_forward(const dpd_plan *P, const dpd_plan *A, const dpd_plan *B, const void *x,
                                  const void *z, const void *grad_y, int64_t rows, int64_t n, int64_t ld,
                                  float scale);

// The one-pass forward of the learning step (dpd_transmit.hip): launches it
// with the plan's coefficients, or with the K device coefficients coeffs_dev
// (each block precombines them itself), loss partials into `partials`; *nblk
// receives the number of partials written.  Arguments already validated.
hipError_t launch_transmit_forward(const dpd_plan *P, const dpd_plan *A, const dpd_plan *B, hipStream_t hs,
                                   const void *coeffs_dev, const void *x, void *z, void *grad_y, int64_t rows,
                                   int64_t n, int64_t ld, float scale, float *partials, int *nblk);
hipError_t launch_bwd_finalize(const float *partials, int nblk, const CoefMap &map, float2 *grad_coeffs,
                               hipStream_t st);

}  // namespace dpd
