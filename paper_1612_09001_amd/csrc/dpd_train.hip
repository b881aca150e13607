// Training helpers: the loss of the coefficient-learning step and an Adam
// update, so that a whole gradient step runs in libdpd's kernels.
//   loss  E = (1/n) sum_t |s*y_t - x_t|^2   (s: 1/PA gain), with
//         dE/dRe y + j dE/dIm y = (2 s / n) (s*y - x);
//   Adam  (Kingma & Ba) on real parameters; complex parameters are their
//         interleaved real and imaginary parts.
// The loss reduction is deterministic: fixed grid, fixed in-block tree, one
// partial per block, then a fixed-order FP64 sum of the partials.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "dpd.h"
#include "dpd_cascade.h"
#include "dpd_internal.h"
#include "dpd_plan.h"

#define DPD_EXPORT extern "C" __attribute__((visibility("default")))

namespace dpd {


// Chunks of 2 kBlock samples: block b takes chunks b, b + grid, ... (the
// blocks running together sweep memory in order), two samples per lane with
// 16-byte accesses when every buffer is 16-byte aligned.  Fixed assignment and
// order: deterministic.
__global__ void __launch_bounds__(kBlock) loss_kernel(const float2 *__restrict__ y, const float2 *__restrict__ x,
                                                      int64_t n, float s, float gscale, float2 *__restrict__ gy,
                                                      float *__restrict__ partials, int vec)
{
    __shared__ double red[kBlock];
    constexpr int64_t CH = 2 * kBlock;
    LossSum ls;
    const auto one = [&](float2 a, float2 b) {
        const float rr = __builtin_fmaf(s, a.x, -b.x), ri = __builtin_fmaf(s, a.y, -b.y);
        ls.f = __builtin_fmaf(rr, rr, __builtin_fmaf(ri, ri, ls.f));
        return make_float2(gscale * rr, gscale * ri);
    };
    for (int64_t c0 = (int64_t)blockIdx.x * CH; c0 < n; c0 += (int64_t)gridDim.x * CH) {
        const int64_t t = c0 + 2 * (int64_t)threadIdx.x;
        if (vec && t + 1 < n) {
            const float4 a = *reinterpret_cast<const float4 *>(y + t);
            const float4 b = *reinterpret_cast<const float4 *>(x + t);
            const float2 g0 = one(make_float2(a.x, a.y), make_float2(b.x, b.y));
            const float2 g1 = one(make_float2(a.z, a.w), make_float2(b.z, b.w));
            if (gy != nullptr) *reinterpret_cast<float4 *>(gy + t) = make_float4(g0.x, g0.y, g1.x, g1.y);
        } else {
#pragma unroll
            for (int i = 0; i < 2; ++i)
                if (t + i < n) {
                    const float2 g0 = one(y[t + i], x[t + i]);
                    if (gy != nullptr) gy[t + i] = g0;
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
    if (threadIdx.x == 0) partials[blockIdx.x] = (float)red[0];
}

// FP64 sum of the block partials: thread t takes partials t, t + 256, ... in
// order, then the DPP lane sum of each wave and the four waves in order
// (bitwise reproducible for a given partial count).
__global__ void __launch_bounds__(kBlock) loss_finalize(const float *__restrict__ partials, int nblk, double inv_n,
                                                        float *__restrict__ loss)
{
    __shared__ double red[kBlock / 64];
    const double u = loss_block_total(partials, nblk, red);
    if (threadIdx.x == 0) *loss = (float)(u * inv_n);
}

__global__ void __launch_bounds__(kBlock) adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                      float *__restrict__ m, float *__restrict__ v, int64_t count,
                                                      float lr, float b1, float b2, float eps, float bc1, float bc2)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
        adam_one(p[i], g[i], m[i], v[i], lr, b1, b2, eps, bc1, bc2);
}

}  // namespace dpd

using namespace dpd;

namespace dpd {

// ----------------------------------------------------------- cascade ---
// A transmitter model of two APH stages, u = A(z) with A memoryless (one tap:
// I/Q imbalance, LO leakage, static nonlinearity) and y = B(u) (a PA with
// memory), fused with the loss above.  One thread takes four consecutive
// samples of a row; the L_B - 1 values of u before them are recomputed from
// z (memoryless A), read from the neighbouring threads' cache lines, so u is
// never stored.  Stage B sees zero input before each row start.

constexpr int kCasQ = 4;   // samples per thread

struct CasParams {
    const float *A;          // precombined table of stage A (L = 1)
    const float *B;          // precombined table of stage B
    int NIA;                 // power levels of A
    const float2 *z, *x;     // rows x n at stride ld
    const float2 *gy;        // backward: dE/dy
    float2 *out;             // forward: dE/dy; backward: dE/dz
    int64_t rows, n, ld, qpr;   // qpr = ceil(n / 4) quads per row
    float scale, gscale;
    float *partials;         // forward: one loss partial per block
    int vec;                 // rows start 16-byte aligned: whole quads use 16-byte accesses
};


// Both tables into registers, once per thread.
template <int NIB, int LB>
__device__ __forceinline__ void cas_tables(const CasParams &p, float (&ta)[kCasTA], float (&tb)[4 * LB * NIB + 2])
{
#pragma unroll
    for (int e = 0; e < kCasTA; ++e) ta[e] = e < 4 * p.NIA + 2 ? p.A[e] : 0.f;
#pragma unroll
    for (int e = 0; e < 4 * LB * NIB + 2; ++e) tb[e] = p.B[e];
}

// Forward: E partials and dE/dy.
template <int NIB, int LB>
__global__ void __launch_bounds__(kBlock) cascade_fwd_kernel(CasParams p)
{
    constexpr int W = kCasQ + LB - 1;
    __shared__ double red[kBlock];
    float ta[kCasTA], tb[4 * LB * NIB + 2];
    cas_tables<NIB, LB>(p, ta, tb);
    LossSum ls;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t q0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    CasWalk wk(q0, stride, p.qpr);
    for (; wk.row < p.rows; wk.next(p.qpr)) {
        const int64_t m0 = wk.k * kCasQ;
        const float2 *zr = p.z + wk.row * p.ld;
        const float2 *xr = p.x + wk.row * p.ld;
        float2 *gr = p.out + wk.row * p.ld;
        // z over the window m0 - (LB-1) .. m0 + 3; 16-byte loads inside the row
        const bool vec = p.vec && m0 + kCasQ <= p.n;
        float2 zw[W], xv[kCasQ];
        if (vec) {
            const float4 a0 = reinterpret_cast<const float4 *>(zr + m0)[0];
            const float4 a1 = reinterpret_cast<const float4 *>(zr + m0)[1];
            zw[LB - 1] = make_float2(a0.x, a0.y);
            zw[LB] = make_float2(a0.z, a0.w);
            zw[LB + 1] = make_float2(a1.x, a1.y);
            zw[LB + 2] = make_float2(a1.z, a1.w);
            const float4 b0 = reinterpret_cast<const float4 *>(xr + m0)[0];
            const float4 b1 = reinterpret_cast<const float4 *>(xr + m0)[1];
            xv[0] = make_float2(b0.x, b0.y);
            xv[1] = make_float2(b0.z, b0.w);
            xv[2] = make_float2(b1.x, b1.y);
            xv[3] = make_float2(b1.z, b1.w);
        } else {
#pragma unroll
            for (int i = 0; i < kCasQ; ++i) {
                zw[LB - 1 + i] = cas_load(zr, m0 + i, p.n);
                xv[i] = cas_load(xr, m0 + i, p.n);
            }
        }
#pragma unroll
        for (int w = 0; w < LB - 1; ++w) zw[w] = cas_load(zr, m0 - (LB - 1) + w, p.n);
        // u = A(z); zero before the row start (stage B's zero history) and past its end
        float2 u[W];
        float sw[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int64_t m = m0 - (LB - 1) + w;
            u[w] = (m >= 0 && m < p.n) ? cas_stage_a(ta, p.NIA, zw[w]) : make_float2(0.f, 0.f);
            sw[w] = __builtin_fmaf(u[w].x, u[w].x, u[w].y * u[w].y);
        }
        float2 g[kCasQ];
#pragma unroll
        for (int i = 0; i < kCasQ; ++i) {
            float yr = tb[4 * LB * NIB], yi = tb[4 * LB * NIB + 1];
#pragma unroll
            for (int k = 0; k < LB; ++k) {
                const int w = i + (LB - 1) - k;
                const float *t = tb + 4 * NIB * k;
                float w00 = t[4 * (NIB - 1)], w01 = t[4 * (NIB - 1) + 1];
                float w10 = t[4 * (NIB - 1) + 2], w11 = t[4 * (NIB - 1) + 3];
#pragma unroll
                for (int j = NIB - 2; j >= 0; --j) {
                    w00 = __builtin_fmaf(w00, sw[w], t[4 * j + 0]);
                    w01 = __builtin_fmaf(w01, sw[w], t[4 * j + 1]);
                    w10 = __builtin_fmaf(w10, sw[w], t[4 * j + 2]);
                    w11 = __builtin_fmaf(w11, sw[w], t[4 * j + 3]);
                }
                yr = __builtin_fmaf(w00, u[w].x, __builtin_fmaf(w01, u[w].y, yr));
                yi = __builtin_fmaf(w10, u[w].x, __builtin_fmaf(w11, u[w].y, yi));
            }
            const bool in = m0 + i < p.n;
            const float rr = in ? __builtin_fmaf(p.scale, yr, -xv[i].x) : 0.f;
            const float ri = in ? __builtin_fmaf(p.scale, yi, -xv[i].y) : 0.f;
            ls.f = __builtin_fmaf(rr, rr, __builtin_fmaf(ri, ri, ls.f));
            g[i] = make_float2(p.gscale * rr, p.gscale * ri);
        }
        if (vec) {
            reinterpret_cast<float4 *>(gr + m0)[0] = make_float4(g[0].x, g[0].y, g[1].x, g[1].y);
            reinterpret_cast<float4 *>(gr + m0)[1] = make_float4(g[2].x, g[2].y, g[3].x, g[3].y);
        } else {
#pragma unroll
            for (int i = 0; i < kCasQ; ++i)
                if (m0 + i < p.n) gr[m0 + i] = g[i];
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

// Backward: dE/dz = A'(z)^T B'(u)^T dE/dy with u = A(z) recomputed.
template <int NIB, int LB>
__global__ void __launch_bounds__(kBlock) cascade_bwd_kernel(CasParams p)
{
    constexpr int W = kCasQ + LB - 1;
    float ta[kCasTA], tb[4 * LB * NIB + 2];
    cas_tables<NIB, LB>(p, ta, tb);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t q0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    CasWalk wk(q0, stride, p.qpr);
    for (; wk.row < p.rows; wk.next(p.qpr)) {
        const int64_t m0 = wk.k * kCasQ;
        const float2 *zr = p.z + wk.row * p.ld;
        const float2 *gyr = p.gy + wk.row * p.ld;
        float2 *out = p.out + wk.row * p.ld;
        const bool vec = p.vec && m0 + kCasQ <= p.n;
        float2 zv[kCasQ], g[W];   // g: dE/dy at m0 .. m0 + 3 + LB - 1 (zero past the row end)
        if (vec) {
            const float4 a0 = reinterpret_cast<const float4 *>(zr + m0)[0];
            const float4 a1 = reinterpret_cast<const float4 *>(zr + m0)[1];
            zv[0] = make_float2(a0.x, a0.y);
            zv[1] = make_float2(a0.z, a0.w);
            zv[2] = make_float2(a1.x, a1.y);
            zv[3] = make_float2(a1.z, a1.w);
            const float4 b0 = reinterpret_cast<const float4 *>(gyr + m0)[0];
            const float4 b1 = reinterpret_cast<const float4 *>(gyr + m0)[1];
            g[0] = make_float2(b0.x, b0.y);
            g[1] = make_float2(b0.z, b0.w);
            g[2] = make_float2(b1.x, b1.y);
            g[3] = make_float2(b1.z, b1.w);
        } else {
#pragma unroll
            for (int i = 0; i < kCasQ; ++i) {
                zv[i] = cas_load(zr, m0 + i, p.n);
                g[i] = cas_load(gyr, m0 + i, p.n);
            }
        }
#pragma unroll
        for (int w = kCasQ; w < W; ++w) g[w] = cas_load(gyr, m0 + w, p.n);
        float2 res[kCasQ];
#pragma unroll
        for (int i = 0; i < kCasQ; ++i) {
            const float2 uv = cas_stage_a(ta, p.NIA, zv[i]);
            const float2 gu = cas_b_adjoint<NIB, LB>(tb, g + i, uv);
            res[i] = cas_a_adjoint(ta, p.NIA, zv[i], gu);
        }
        if (vec) {
            reinterpret_cast<float4 *>(out + m0)[0] = make_float4(res[0].x, res[0].y, res[1].x, res[1].y);
            reinterpret_cast<float4 *>(out + m0)[1] = make_float4(res[2].x, res[2].y, res[3].x, res[3].y);
        } else {
#pragma unroll
            for (int i = 0; i < kCasQ; ++i)
                if (m0 + i < p.n) out[m0 + i] = res[i];
        }
    }
}

constexpr int kCasMaxNI = 4;   // stage B: orders up to 7
constexpr int kCasMaxL = 4;    // stage B: up to 4 taps

typedef void (*CasKernel)(CasParams);

template <int NI, int L>
struct CasEntry {
    static void fill(CasKernel (&f)[kCasMaxNI][kCasMaxL], CasKernel (&b)[kCasMaxNI][kCasMaxL])
    {
        f[NI - 1][L - 1] = &cascade_fwd_kernel<NI, L>;
        b[NI - 1][L - 1] = &cascade_bwd_kernel<NI, L>;
        if constexpr (L < kCasMaxL)
            CasEntry<NI, L + 1>::fill(f, b);
        else if constexpr (NI < kCasMaxNI)
            CasEntry<NI + 1, 1>::fill(f, b);
    }
};

struct CasTable {
    CasKernel fwd[kCasMaxNI][kCasMaxL];
    CasKernel bwd[kCasMaxNI][kCasMaxL];
    CasTable() { CasEntry<1, 1>::fill(fwd, bwd); }
};

static const CasTable &cas_table()
{
    static const CasTable t;
    return t;
}

static dpd_status cas_check(const dpd_plan *A, const dpd_plan *B, const void *p0, const void *p1, const void *out,
                            int64_t rows, int64_t n, int64_t ld)
{
    if (A == nullptr || B == nullptr) return DPD_EINVAL;
    if (A->map.L != 1) return DPD_EINVAL;
    if (B->map.NI > kCasMaxNI || B->map.L > kCasMaxL) return DPD_EUNSUPPORTED;
    if (rows < 0 || n < 0 || (rows > 1 && ld < n)) return DPD_EINVAL;
    if (rows == 0 || n == 0) return DPD_OK;
    if (p0 == nullptr || p1 == nullptr || out == nullptr) return DPD_EINVAL;
    for (const void *q : {p0, p1, out})
        if ((uintptr_t)q % 8 != 0) return DPD_EINVAL;
    const size_t span = (size_t)(((rows - 1) * (rows > 1 ? ld : n) + n) * (int64_t)sizeof(float2));
    const auto lap = [&](const void *a, const void *b) {
        const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
        return x < y + span && y < x + span;
    };
    if (lap(out, p0) || lap(out, p1)) return DPD_EINVAL;
    return DPD_OK;
}

hipError_t launch_loss_finalize(const float *partials, int nblk, double inv_n, float *loss, hipStream_t st)
{
    hipLaunchKernelGGL(loss_finalize, dim3(1), dim3(kBlock), 0, st, partials, nblk, inv_n, loss);
    return hipGetLastError();
}

static int cas_grid(int64_t total)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>(kLossBlocks, (total + kBlock - 1) / kBlock));
}

}  // namespace dpd

using namespace dpd;

DPD_EXPORT dpd_status dpd_cascade_loss_grad(const dpd_plan *A, const dpd_plan *B, void *stream, const void *z,
                                            const void *x, int64_t rows, int64_t n, int64_t ld, float scale,
                                            float *loss_dev, void *grad_y, void *ws, size_t ws_bytes)
{
    dpd_status st = cas_check(A, B, z, x, grad_y, rows, n, ld);
    if (st != DPD_OK) return st;
    if (ws == nullptr || ws_bytes < kLossBlocks * sizeof(float) || (uintptr_t)ws % 4 != 0) return DPD_EINVAL;
    if (!std::isfinite(scale)) return DPD_EINVAL;
    const hipStream_t hs = (hipStream_t)stream;
    const int64_t N = rows * n;
    int nblk = 0;
    if (N > 0) {
        CasParams p;
        p.A = A->d_table;
        p.B = B->d_table;
        p.NIA = A->map.NI;
        p.z = (const float2 *)z;
        p.x = (const float2 *)x;
        p.gy = nullptr;
        p.out = (float2 *)grad_y;
        p.rows = rows;
        p.n = n;
        p.ld = rows > 1 ? ld : n;
        p.qpr = (n + kCasQ - 1) / kCasQ;
        p.scale = scale;
        p.gscale = (float)(2.0 * scale / (double)N);
        p.partials = (float *)ws;
        p.vec = ((uintptr_t)z % 16 == 0 && (uintptr_t)x % 16 == 0 && (uintptr_t)grad_y % 16 == 0 &&
                 (rows == 1 || ld % 2 == 0)) ? 1 : 0;
        nblk = cas_grid(rows * p.qpr);
        hipLaunchKernelGGL(cas_table().fwd[B->map.NI - 1][B->map.L - 1], dim3(nblk), dim3(kBlock), 0, hs, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e);
    }
    if (loss_dev != nullptr) {
        hipLaunchKernelGGL(loss_finalize, dim3(1), dim3(kBlock), 0, hs, (const float *)ws, nblk,
                           N > 0 ? 1.0 / (double)N : 0.0, loss_dev);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e);
    }
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_cascade_backward(const dpd_plan *A, const dpd_plan *B, void *stream, const void *z,
                                           const void *grad_y, void *grad_z, int64_t rows, int64_t n, int64_t ld)
{
    dpd_status st = cas_check(A, B, z, grad_y, grad_z, rows, n, ld);
    if (st != DPD_OK || rows == 0 || n == 0) return st;
    CasParams p;
    p.A = A->d_table;
    p.B = B->d_table;
    p.NIA = A->map.NI;
    p.z = (const float2 *)z;
    p.x = nullptr;
    p.gy = (const float2 *)grad_y;
    p.out = (float2 *)grad_z;
    p.rows = rows;
    p.n = n;
    p.ld = rows > 1 ? ld : n;
    p.qpr = (n + kCasQ - 1) / kCasQ;
    p.scale = 0.f;
    p.gscale = 0.f;
    p.partials = nullptr;
    p.vec = ((uintptr_t)z % 16 == 0 && (uintptr_t)grad_y % 16 == 0 && (uintptr_t)grad_z % 16 == 0 &&
             (rows == 1 || ld % 2 == 0)) ? 1 : 0;
    hipLaunchKernelGGL(cas_table().bwd[B->map.NI - 1][B->map.L - 1], dim3(cas_grid(rows * p.qpr)), dim3(kBlock), 0,
                       (hipStream_t)stream, p);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}

DPD_EXPORT dpd_status dpd_loss_ws_size(int64_t n, size_t *bytes)
{
    if (n < 0 || bytes == nullptr) return DPD_EINVAL;
    *bytes = kLossBlocks * sizeof(float);
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_loss_grad(void *stream, const void *y, const void *x, int64_t n, float scale,
                                    float *loss_dev, void *grad_y, void *ws, size_t ws_bytes)
{
    if (n < 0 || (n > 0 && (y == nullptr || x == nullptr))) return DPD_EINVAL;
    if (ws == nullptr || ws_bytes < kLossBlocks * sizeof(float) || (uintptr_t)ws % 4 != 0) return DPD_EINVAL;
    for (const void *q : {y, x, (const void *)grad_y})
        if ((uintptr_t)q % 8 != 0) return DPD_EINVAL;
    const hipStream_t st = (hipStream_t)stream;
    int nblk = 0;
    if (n > 0) {
        nblk = (int)std::min<int64_t>(kLossBlocks, (n + kBlock - 1) / kBlock);
        const float gscale = (float)(2.0 * scale / (double)n);
        const int vec = ((uintptr_t)y % 16 == 0 && (uintptr_t)x % 16 == 0 && (uintptr_t)grad_y % 16 == 0) ? 1 : 0;
        hipLaunchKernelGGL(loss_kernel, dim3(nblk), dim3(kBlock), 0, st, (const float2 *)y, (const float2 *)x, n,
                           scale, gscale, (float2 *)grad_y, (float *)ws, vec);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e);
    }
    if (loss_dev != nullptr) {
        hipLaunchKernelGGL(loss_finalize, dim3(1), dim3(kBlock), 0, st, (const float *)ws, nblk,
                           n > 0 ? 1.0 / (double)n : 0.0, loss_dev);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e);
    }
    return DPD_OK;
}

DPD_EXPORT dpd_status dpd_adam_step(void *stream, float *params, const float *grads, float *m, float *v,
                                    int64_t count, int32_t step, float lr, float beta1, float beta2, float eps)
{
    if (count < 0 || step < 1) return DPD_EINVAL;
    if (count > 0 && (params == nullptr || grads == nullptr || m == nullptr || v == nullptr)) return DPD_EINVAL;
    if (count == 0) return DPD_OK;
    const float bc1 = (float)(1.0 - std::pow((double)beta1, step));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, step));
    const int64_t blocks = std::min<int64_t>((count + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(adam_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, (hipStream_t)stream, params, grads, m,
                       v, count, lr, beta1, beta2, eps, bc1, bc2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}
