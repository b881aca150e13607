// Pieces of the transmitter-cascade kernels shared by the training
// translation units (dpd_train.hip, dpd_transmit.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "dpd_internal.h"

namespace dpd {

constexpr int kLossBlocks = 1024;   // loss partials (one per block of the loss kernels)

constexpr int kCasTA = 4 * kMaxNI + 2;   // stage-A table floats held in registers (at most)

// A(z) for one sample (memoryless: c + W(|z|^2) z, W by Horner over NIA levels)
__device__ __forceinline__ float2 cas_stage_a(const float (&T)[kCasTA], int NIA, float2 v)
{
    const float s = __builtin_fmaf(v.x, v.x, v.y * v.y);
    float w00 = 0.f, w01 = 0.f, w10 = 0.f, w11 = 0.f, cr = 0.f, ci = 0.f;
#pragma unroll
    for (int j = kMaxNI - 1; j >= 0; --j) {
        if (j < NIA) {
            w00 = __builtin_fmaf(w00, s, T[4 * j + 0]);
            w01 = __builtin_fmaf(w01, s, T[4 * j + 1]);
            w10 = __builtin_fmaf(w10, s, T[4 * j + 2]);
            w11 = __builtin_fmaf(w11, s, T[4 * j + 3]);
        }
        if (j == NIA) {
            cr = T[4 * j];
            ci = T[4 * j + 1];
        }
    }
    if (NIA == kMaxNI) {
        cr = T[4 * kMaxNI];
        ci = T[4 * kMaxNI + 1];
    }
    return make_float2(__builtin_fmaf(w00, v.x, __builtin_fmaf(w01, v.y, cr)),
                       __builtin_fmaf(w10, v.x, __builtin_fmaf(w11, v.y, ci)));
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

}  // namespace dpd
