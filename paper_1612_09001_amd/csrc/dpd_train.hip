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
#include "dpd_internal.h"
#include "dpd_plan.h"

#define DPD_EXPORT extern "C" __attribute__((visibility("default")))

namespace dpd {

constexpr int kLossBlocks = 1024;

__global__ void __launch_bounds__(kBlock) loss_kernel(const float2 *__restrict__ y, const float2 *__restrict__ x,
                                                      int64_t n, float s, float gscale, float2 *__restrict__ gy,
                                                      float *__restrict__ partials)
{
    __shared__ float red[kBlock];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    float acc = 0.f;
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBlock) {
        const float2 a = y[t], b = x[t];
        const float rr = __builtin_fmaf(s, a.x, -b.x), ri = __builtin_fmaf(s, a.y, -b.y);
        acc = __builtin_fmaf(rr, rr, __builtin_fmaf(ri, ri, acc));
        if (gy != nullptr) gy[t] = make_float2(gscale * rr, gscale * ri);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// FP64 sum of the block partials: thread t takes partials t, t + 256, ... in
// order, then a fixed butterfly in each wave and the four waves in order
// (bitwise reproducible for a given partial count).
__global__ void __launch_bounds__(kBlock) loss_finalize(const float *__restrict__ partials, int nblk, double inv_n,
                                                        float *__restrict__ loss)
{
    __shared__ double red[kBlock / 64];
    double t = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) t += (double)partials[b];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double u = red[0];
        for (int w = 1; w < kBlock / 64; ++w) u += red[w];
        *loss = (float)(u * inv_n);
    }
}

__global__ void __launch_bounds__(kBlock) adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                      float *__restrict__ m, float *__restrict__ v, int64_t count,
                                                      float lr, float b1, float b2, float eps, float bc1, float bc2)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock) {
        const float gi = g[i];
        const float mi = __builtin_fmaf(b1, m[i], (1.f - b1) * gi);
        const float vi = __builtin_fmaf(b2, v[i], (1.f - b2) * gi * gi);
        m[i] = mi;
        v[i] = vi;
        const float denom = __builtin_sqrtf(vi / bc2) + eps;
        p[i] -= (lr / bc1) * mi / denom;
    }
}

}  // namespace dpd

using namespace dpd;

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
        hipLaunchKernelGGL(loss_kernel, dim3(nblk), dim3(kBlock), 0, st, (const float2 *)y, (const float2 *)x, n,
                           scale, gscale, (float2 *)grad_y, (float *)ws);
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
