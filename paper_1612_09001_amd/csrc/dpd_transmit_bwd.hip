// The backward pass of the coefficient-learning step in one kernel: the
// adjoint of the two-stage transmitter model (stage B, the PA with memory, at
// u = A(z); then the memoryless stage A at z) gives dE/dz, and the coefficient
// gradient of the predistorter (Eq. 1 / Algorithm 1 differentiated in its
// coefficients) correlates dE/dz with the basis of x at once:
//     dE/dM_{j,k}[r][c] = sum_m G_{m+k}[r] (s_m^j v_m)[c],   G = dE/dz,
// with v_m = (Re x_m, Im x_m), s_m = |x_m|^2 -- so dE/dz never goes to memory.
// The predistorter's coefficients are not read (the gradient does not depend
// on them).
//
// Rows of whole 256-sample chunks, 16-byte aligned.  Each wave takes a
// contiguous run of chunks of the flattened rows and walks it from its end:
// lane l owns samples 4l .. 4l + 3 of a chunk, computes G there from z and
// dE/dy (dE/dy staged with the LB - 1 samples after the chunk), and pairs G at
// m .. m + L - 1 with the basis at m, so the L - 1 values of G after the chunk
// are the first ones of the chunk handled just before (carried in registers),
// zero past the row end, and -- for the first chunk of a run inside a row --
// evaluated directly by L - 1 lanes.  The per-sample arithmetic of G is that
// of dpd_cascade_backward (bitwise the same values).  The coefficient-gradient
// accumulation, its fixed-order reduction to one FP32 partial per block and
// the FP64 finalisation are those of dpd_backward.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>

#include "dpd.h"
#include "dpd_bwd_kernels.h"
#include "dpd_cascade.h"
#include "dpd_plan.h"

#define DPD_EXPORT extern "C" __attribute__((visibility("default")))

namespace dpd {

constexpr int kTbNIB = 3, kTbLB = 3;   // stage B of the one-pass form: orders {1,3,5}, 3 taps
constexpr int kTbMaxNI = 5;            // predistorter: orders up to 9
constexpr int kTbMaxL = kSpecL;        // predistorter: up to 8 taps
constexpr int kTbChunk = 64 * kBwdS;   // samples per wave chunk

struct TbParams {
    const float *A, *B;       // transmitter stage tables
    const float2 *x, *z, *gy; // rows x n at stride ld
    float2 *gz;               // dE/dz out (nullptr: not written)
    float *partials;          // [gridDim.x][4 L NI + 2]
    int64_t rows, n, ld, tpr; // tpr = n / chunk
    int32_t *step;            // learning-step counter advanced by one (nullptr: none)
};

template <int NI, int L>
__global__ void __launch_bounds__(kBlock) transmit_bwd_kernel(TbParams p)
{
    constexpr int NIB = kTbNIB, LB = kTbLB;
    constexpr int S = kBwdS, C = kTbChunk, NV = S / 2, WAVES = kBlock / 64;
    constexpr int W = S + L - 1;        // G window of a lane
    constexpr int HG = L - 1;           // G after the chunk
    constexpr int HY = LB - 1;          // dE/dy after the chunk
    constexpr int E = 4 * L * NI + 2;
    constexpr int GSLOTS = C + HG + (C + HG) / S + 1;
    constexpr int YSLOTS = C + HY + (C + HY) / S + 1;
    constexpr int XSLOTS = C + C / S;
    __shared__ __align__(16) float2 gs[WAVES][GSLOTS];
    __shared__ __align__(16) float2 ys[WAVES][YSLOTS];
    __shared__ __align__(16) float2 xsh[WAVES][XSLOTS];
    __shared__ __align__(16) float2 zsh[WAVES][XSLOTS];
    __shared__ double red[WAVES * E];   // per-wave FP64 totals of the coefficient gradient

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    float ta[kCasTA], tb[4 * LB * NIB + 2];
#pragma unroll
    for (int e = 0; e < kCasTA; ++e) ta[e] = e < 6 ? p.A[e] : 0.f;
#pragma unroll
    for (int e = 0; e < 4 * LB * NIB + 2; ++e) tb[e] = p.B[e];
    float2 *G = gs[wv];
    float2 *Y = ys[wv];
    float2 *X = xsh[wv];
    float2 *Z = zsh[wv];
    auto slot = [](int d) { return d + d / S; };

    float acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0.f;
    // per-lane FP32 sums over at most kBwdFlush chunks, then into the wave's
    // FP64 totals, entry 64 g + l in lane l of tot[g] (the rounding error does
    // not grow with the batch size)
    constexpr int NGT = (E + 63) / 64;
    double tot[NGT];
#pragma unroll
    for (int g = 0; g < NGT; ++g) tot[g] = 0.0;
    auto flush = [&]() {
        wave_sums_into<E>(acc, tot, lane);
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = 0.f;
    };

    // G at sample m of a row from z and dE/dy (zero past the row end): the
    // arithmetic of dpd_cascade_backward
    auto g_at = [&](const float2 *zr, const float2 *yr, int64_t m) {
        const float2 zv = cas_load(zr, m, p.n);
        float2 g[LB];
#pragma unroll
        for (int k = 0; k < LB; ++k) g[k] = cas_load(yr, m + k, p.n);
        const float2 uv = cas_stage_a(ta, 1, zv);
        const float2 gu = cas_b_adjoint<NIB, LB>(tb, g, uv);
        return cas_a_adjoint(ta, 1, zv, gu);
    };

    struct Regs {
        float4 z[NV], y[NV], x[NV];
        float2 yh;   // dE/dy at t0 + C + lane (lanes < HY; zero past the row end)
    };
    auto load = [&](Regs &R, int64_t row, int64_t t0) {
        __builtin_amdgcn_s_setprio(2);   // the prefetch at raised wave priority
        const int64_t base = row * p.ld + t0;
        const v4f *z4 = reinterpret_cast<const v4f *>(p.z + base);
        const v4f *y4 = reinterpret_cast<const v4f *>(p.gy + base);
        const v4f *x4 = reinterpret_cast<const v4f *>(p.x + base);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const v4f a = __builtin_nontemporal_load(z4 + lane + 64 * i);
            R.z[i] = make_float4(a.x, a.y, a.z, a.w);
        }
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const v4f a = __builtin_nontemporal_load(y4 + lane + 64 * i);
            R.y[i] = make_float4(a.x, a.y, a.z, a.w);
        }
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const v4f a = __builtin_nontemporal_load(x4 + lane + 64 * i);
            R.x[i] = make_float4(a.x, a.y, a.z, a.w);
        }
        // the LB - 1 values after the chunk: inside the row unless it is the row's last chunk
        const int hl = lane < HY ? lane : HY - 1;
        const bool in = t0 + C < p.n;
        const float2 v = p.gy[row * p.ld + (in ? t0 + C + hl : t0)];
        R.yh = in ? v : make_float2(0.f, 0.f);
        __builtin_amdgcn_s_setprio(0);
    };
    auto stage = [&](const Regs &R) {
        wave_lds_order();   // the previous chunk's LDS reads are done
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int j = 2 * (lane + 64 * i);
            Z[slot(j)] = make_float2(R.z[i].x, R.z[i].y);
            Z[slot(j) + 1] = make_float2(R.z[i].z, R.z[i].w);
            Y[slot(j)] = make_float2(R.y[i].x, R.y[i].y);
            Y[slot(j) + 1] = make_float2(R.y[i].z, R.y[i].w);
            X[slot(j)] = make_float2(R.x[i].x, R.x[i].y);
            X[slot(j) + 1] = make_float2(R.x[i].z, R.x[i].w);
        }
        if (lane < HY) Y[slot(C + lane)] = R.yh;
        wave_lds_order();
    };
    // one staged chunk; `carry` holds G at t0 + C + lane (lanes < HG) and
    // leaves with G at t0 + lane, the values the chunk before needs
    auto compute = [&](int64_t row, int64_t t0, float2 &carry) {
        float2 gz[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const float2 zv = Z[slot(lane * S + i)];
            float2 g[LB];
#pragma unroll
            for (int k = 0; k < LB; ++k) g[k] = Y[slot(lane * S + i + k)];
            const float2 uv = cas_stage_a(ta, 1, zv);
            const float2 gu = cas_b_adjoint<NIB, LB>(tb, g, uv);
            gz[i] = cas_a_adjoint(ta, 1, zv, gu);
        }
#pragma unroll
        for (int i = 0; i < S; ++i) G[slot(lane * S + i)] = gz[i];
        if (HG > 0 && lane < HG) G[slot(C + lane)] = carry;
        wave_lds_order();
        if (HG > 0) {
            const float2 c = G[slot(lane < HG ? lane : 0)];
            carry = lane < HG ? c : make_float2(0.f, 0.f);
        }
        float ga[W], gb[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const float2 g = G[slot(lane * S + w)];
            ga[w] = g.x;
            gb[w] = g.y;
        }
        float va[S], vb[S], sq[S], pw[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const float2 v = X[slot(lane * S + i)];
            va[i] = v.x;
            vb[i] = v.y;
            sq[i] = __builtin_fmaf(v.x, v.x, v.y * v.y);
            pw[i] = 1.f;
        }
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            float ba[S], bb[S];
#pragma unroll
            for (int i = 0; i < S; ++i) {
                ba[i] = pw[i] * va[i];
                bb[i] = pw[i] * vb[i];
            }
#pragma unroll
            for (int k = 0; k < L; ++k) {
#pragma unroll
                for (int i = 0; i < S; ++i) {
                    const float a = ga[i + k], b = gb[i + k];
                    float *u = &acc[4 * (k * NI + j)];
                    u[0] = __builtin_fmaf(a, ba[i], u[0]);
                    u[1] = __builtin_fmaf(a, bb[i], u[1]);
                    u[2] = __builtin_fmaf(b, ba[i], u[2]);
                    u[3] = __builtin_fmaf(b, bb[i], u[3]);
                }
            }
#pragma unroll
            for (int i = 0; i < S; ++i) pw[i] *= sq[i];
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
            acc[E - 2] += ga[i];
            acc[E - 1] += gb[i];
        }
        if (p.gz != nullptr) {
            // G back through LDS so every store instruction writes 1 KiB
            v4f *o4 = reinterpret_cast<v4f *>(p.gz + row * p.ld + t0);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int j = 2 * (lane + 64 * i);
                const float2 u = G[slot(j)], w = G[slot(j) + 1];
                const v4f v = {u.x, u.y, w.x, w.y};
                __builtin_nontemporal_store(v, o4 + lane + 64 * i);
            }
        }
    };

    const int64_t total = p.rows * p.tpr;
    const int64_t nw = (int64_t)gridDim.x * WAVES;
    const int64_t gw = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * WAVES + wv;
    const int64_t per = (total + nw - 1) / nw;
    const int64_t c_begin = gw * per < total ? gw * per : total;
    const int64_t c_end = c_begin + per < total ? c_begin + per : total;
    // the learning step's counter (read by the finalisation launch after this one)
    if (p.step != nullptr && blockIdx.x == 0 && tid == 0) *p.step += 1;
    if (c_begin < c_end) {
        // the run's last chunk first
        int64_t row = (c_end - 1) / p.tpr;
        int64_t k = (c_end - 1) - row * p.tpr;
        float2 carry = make_float2(0.f, 0.f);
        if (HG > 0) {
            // G after the chunk: zero past the row end, else evaluated here
            const int64_t m = (k + 1) * C + (lane < HG ? lane : 0);
            const float2 v = g_at(p.z + row * p.ld, p.gy + row * p.ld, m);
            carry = lane < HG ? v : make_float2(0.f, 0.f);
        }
        Regs R;
        load(R, row, k * C);
        stage(R);
        for (int64_t left = c_end - c_begin; left > 1; --left) {
            const int64_t crow = row, ck = k;
            if (k == 0) {
                --row;
                k = p.tpr - 1;
            } else {
                --k;
            }
            load(R, row, k * C);
            compute(crow, ck * C, carry);
            if (ck == 0) carry = make_float2(0.f, 0.f);   // the chunk before ends a row
            stage(R);
            if (((c_end - c_begin - left) & (kBwdFlush - 1)) == kBwdFlush - 1) flush();
        }
        compute(row, k * C, carry);
    }

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

typedef void (*TbKernel)(TbParams);

template <int NI, int L>
struct TbEntry {
    static void fill(TbKernel (&f)[kTbMaxNI][kTbMaxL])
    {
        f[NI - 1][L - 1] = &transmit_bwd_kernel<NI, L>;
        if constexpr (L < kTbMaxL)
            TbEntry<NI, L + 1>::fill(f);
        else if constexpr (NI < kTbMaxNI)
            TbEntry<NI + 1, 1>::fill(f);
    }
};

struct TbTable {
    TbKernel k[kTbMaxNI][kTbMaxL];
    TbTable() { TbEntry<1, 1>::fill(k); }
};

static const TbTable &tb_table()
{
    static const TbTable t;
    return t;
}

int num_cus();

static int tb_occupancy(int NI, int L)
{
    static std::atomic<int> cache[kTbMaxNI][kTbMaxL] = {};
    int v = cache[NI - 1][L - 1].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, (const void *)tb_table().k[NI - 1][L - 1], kBlock, 0) !=
                hipSuccess ||
            v < 1)
            v = 1;
        cache[NI - 1][L - 1].store(v, std::memory_order_relaxed);
    }
    return v;
}

// The one-pass backward into coefficient-gradient partials; *nblk receives
// how many blocks wrote them.  Shapes already checked (whole chunks, aligned).
__global__ void step_advance(int32_t *step) { *step += 1; }

static hipError_t launch_tb(const dpd_plan *P, const dpd_plan *A, const dpd_plan *B, hipStream_t hs, const void *x,
                            const void *z, const void *grad_y, void *grad_z, float *partials, int64_t rows,
                            int64_t n, int64_t rs, int *nblk, int32_t *step = nullptr)
{
    *nblk = 0;
    if (rows * n == 0) {
        if (step == nullptr) return hipSuccess;
        hipLaunchKernelGGL(step_advance, dim3(1), dim3(1), 0, hs, step);
        return hipGetLastError();
    }
    TbParams p;
    p.step = step;
    p.A = A->d_table;
    p.B = B->d_table;
    p.x = (const float2 *)x;
    p.z = (const float2 *)z;
    p.gy = (const float2 *)grad_y;
    p.gz = (float2 *)grad_z;
    p.partials = partials;
    p.rows = rows;
    p.n = n;
    p.ld = rs;
    p.tpr = n / kTbChunk;
    // one round of resident blocks, at most two per CU, each wave a run of chunks
    const int NI = P->map.NI, L = P->map.L;
    const int64_t cap = (int64_t)num_cus() * std::min(tb_occupancy(NI, L), 2);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cap, (rows * p.tpr + 3) / 4));
    hipLaunchKernelGGL(tb_table().k[NI - 1][L - 1], dim3(grid), dim3(kBlock), 0, hs, p);
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) *nblk = grid;
    return e;
}

static bool tb_shapes_ok(const dpd_plan *P, const dpd_plan *A, const dpd_plan *B, const void *x, const void *z,
                         const void *grad_y, const void *grad_z, int64_t n, int64_t rs)
{
    const bool stages = A->map.NI == 1 && B->map.NI == kTbNIB && B->map.L == kTbLB && P->map.NI <= kTbMaxNI &&
                        P->map.L <= kTbMaxL;
    const bool aligned = (uintptr_t)x % 16 == 0 && (uintptr_t)z % 16 == 0 && (uintptr_t)grad_y % 16 == 0 &&
                         (uintptr_t)grad_z % 16 == 0 && rs % 2 == 0;
    return stages && aligned && n % kTbChunk == 0;
}

// Learning-step finalisation in one launch: blocks 0 .. L NI sum the
// coefficient-gradient partials of their table entry in FP64 (as dpd_backward
// does), write the gradients (grad_coeffs may be NULL) and apply Adam to the
// coefficients they belong to (as dpd_adam_step does: each coefficient has
// exactly one entry); block L NI + 1 sums the loss partials.
__global__ void __launch_bounds__(kBlock) learn_finalize(const float *__restrict__ dc, int nblk, CoefMap map,
                                                         const float *__restrict__ lp, int nloss, double inv_n,
                                                         float *__restrict__ loss, float2 *__restrict__ gcoef,
                                                         float *__restrict__ params, float *__restrict__ m,
                                                         float *__restrict__ v, float lr, float b1, float b2,
                                                         float eps, float bc1, float bc2,
                                                         const int32_t *__restrict__ step)
{
    __shared__ double red[kBlock / 64][4];
    if (step != nullptr) {
        // Adam's bias corrections from the device-side step count
        const double t = (double)*step;
        bc1 = (float)(1.0 - pow((double)b1, t));
        bc2 = (float)(1.0 - pow((double)b2, t));
    }
    __shared__ double lred[kBlock / 64];
    const int q = blockIdx.x;
    if (q == map.L * map.NI + 1) {
        const double u = loss_block_total(lp, nloss, lred);
        if (threadIdx.x == 0 && loss != nullptr) *loss = (float)(u * inv_n);
        return;
    }
    double u[4];
    dcoef_block_sums(dc, nblk, map, q, red, u);
    if (threadIdx.x != 0) return;
    int idx[2];
    float2 g[2];
    const int c = dcoef_block_grads(map, q, u, idx, g);
    for (int i = 0; i < c; ++i) {
        if (gcoef != nullptr) gcoef[idx[i]] = g[i];
        const int r = 2 * idx[i];
        adam_one(params[r], g[i].x, m[r], v[r], lr, b1, b2, eps, bc1, bc2);
        adam_one(params[r + 1], g[i].y, m[r + 1], v[r + 1], lr, b1, b2, eps, bc1, bc2);
    }
}

// Workspace of dpd_learn_step: the loss partials, then (256-byte aligned) the
// coefficient-gradient partials.
static size_t learn_loss_bytes() { return ((size_t)kLossBlocks * sizeof(float) + 255) & ~(size_t)255; }

}  // namespace dpd

using namespace dpd;

DPD_EXPORT dpd_status dpd_transmit_backward(const dpd_plan *P, const dpd_plan *A, const dpd_plan *B, void *stream,
                                            const void *x, const void *z, const void *grad_y, void *grad_z,
                                            void *grad_coeffs, int64_t rows, int64_t n, int64_t ld, void *ws,
                                            size_t ws_bytes)
{
    if (P == nullptr || A == nullptr || B == nullptr || grad_coeffs == nullptr) return DPD_EINVAL;
    if (A->map.L != 1) return DPD_EINVAL;
    if (rows < 0 || n < 0 || (rows > 1 && ld < n)) return DPD_EINVAL;
    if (ws == nullptr || ws_bytes < bwd_ws_bytes(P->map) || (uintptr_t)ws % 4 != 0) return DPD_EINVAL;
    if ((uintptr_t)grad_coeffs % 8 != 0) return DPD_EINVAL;
    const int64_t N = rows * n;
    const int64_t rs = rows > 1 ? ld : n;
    if (N > 0) {
        if (x == nullptr || z == nullptr || grad_y == nullptr) return DPD_EINVAL;
        for (const void *q : {x, z, grad_y, (const void *)grad_z})
            if ((uintptr_t)q % 8 != 0) return DPD_EINVAL;
        if (grad_z != nullptr) {
            const size_t span = (size_t)(((rows - 1) * rs + n) * (int64_t)sizeof(float2));
            const auto lap = [&](const void *a, const void *b) {
                const uintptr_t u = (uintptr_t)a, v = (uintptr_t)b;
                return u < v + span && v < u + span;
            };
            if (lap(grad_z, x) || lap(grad_z, z) || lap(grad_z, grad_y)) return DPD_EINVAL;
        }
    }
    const hipStream_t hs = (hipStream_t)stream;
    if (!tb_shapes_ok(P, A, B, x, z, grad_y, grad_z, n, rs)) {
        // other shapes: the two passes, dE/dz through the caller's grad_z
        if (N > 0 && grad_z == nullptr) return DPD_EUNSUPPORTED;
        dpd_status st = dpd_cascade_backward(A, B, stream, z, grad_y, grad_z, rows, n, ld);
        if (st != DPD_OK) return st;
        return dpd_backward(const_cast<dpd_plan *>(P), stream, nullptr, x, grad_z, nullptr, grad_coeffs, rows, n,
                            ld, ws, ws_bytes);
    }
    int nblk = 0;
    hipError_t e = launch_tb(P, A, B, hs, x, z, grad_y, grad_z, (float *)ws, rows, n, rs, &nblk);
    if (e != hipSuccess) return hip_fail(e);
    e = launch_bwd_finalize((const float *)ws, nblk, P->map, (float2 *)grad_coeffs, hs);
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}

DPD_EXPORT dpd_status dpd_learn_step_ws_size(const dpd_plan *P, size_t *bytes)
{
    if (P == nullptr || bytes == nullptr) return DPD_EINVAL;
    *bytes = learn_loss_bytes() + bwd_ws_bytes(P->map);
    return DPD_OK;
}

// The learning step with the Adam step count from the host (step >= 1) or,
// with step_dev, from a device counter the call advances.
static dpd_status learn_step(dpd_plan *P, const dpd_plan *A, const dpd_plan *B, void *stream, void *coeffs_dev,
                             float *adam_m, float *adam_v, int32_t step, int32_t *step_dev, float lr, float beta1,
                             float beta2, float eps, const void *x, void *z, void *grad_y, int64_t rows, int64_t n,
                             int64_t ld, float scale, float *loss_dev, void *grad_coeffs, void *ws, size_t ws_bytes)
{
    dpd_status st = check_transmit_forward(P, A, B, x, z, grad_y, rows, n, ld, scale);
    if (st != DPD_OK) return st;
    if (coeffs_dev == nullptr || adam_m == nullptr || adam_v == nullptr) return DPD_EINVAL;
    if (step_dev == nullptr ? step < 1 : (uintptr_t)step_dev % 4 != 0) return DPD_EINVAL;
    if ((uintptr_t)coeffs_dev % 8 != 0 || (uintptr_t)adam_m % 4 != 0 || (uintptr_t)adam_v % 4 != 0 ||
        (uintptr_t)grad_coeffs % 8 != 0)
        return DPD_EINVAL;
    if (!std::isfinite(lr) || !std::isfinite(beta1) || !std::isfinite(beta2) || !std::isfinite(eps))
        return DPD_EINVAL;
    const size_t need = learn_loss_bytes() + bwd_ws_bytes(P->map);
    if (ws == nullptr || ws_bytes < need || (uintptr_t)ws % 4 != 0) return DPD_EINVAL;
    // the K coefficients, their Adam moments and the gradient output must not overlap
    const size_t kb = (size_t)P->K * sizeof(float2);
    const auto lap = [kb](const void *a, const void *b) {
        const uintptr_t u = (uintptr_t)a, v = (uintptr_t)b;
        return a != nullptr && b != nullptr && u < v + kb && v < u + kb;
    };
    if (lap(coeffs_dev, adam_m) || lap(coeffs_dev, adam_v) || lap(adam_m, adam_v) || lap(grad_coeffs, coeffs_dev) ||
        lap(grad_coeffs, adam_m) || lap(grad_coeffs, adam_v))
        return DPD_EINVAL;
    if (step_dev != nullptr) {
        // nor the step counter any of them
        const auto in = [kb](const void *base, const void *q) {
            const uintptr_t u = (uintptr_t)base, v = (uintptr_t)q;
            return base != nullptr && v + sizeof(int32_t) > u && v < u + kb;
        };
        if (in(coeffs_dev, step_dev) || in(adam_m, step_dev) || in(adam_v, step_dev) || in(grad_coeffs, step_dev))
            return DPD_EINVAL;
    }
    const int64_t rs = rows > 1 ? ld : n;
    if (!tb_shapes_ok(P, A, B, x, z, grad_y, nullptr, n, rs)) return DPD_EUNSUPPORTED;
    const hipStream_t hs = (hipStream_t)stream;
    const int64_t N = rows * n;
    float *lp = (float *)ws;
    float *dc = (float *)((char *)ws + learn_loss_bytes());
    int nloss = 0, nblk = 0;
    hipError_t e = launch_transmit_forward(P, A, B, hs, coeffs_dev, x, z, grad_y, rows, n, ld, scale, lp, &nloss);
    if (e != hipSuccess) return hip_fail(e);
    e = launch_tb(P, A, B, hs, x, z, grad_y, nullptr, dc, rows, n, rs, &nblk, step_dev);
    if (e != hipSuccess) return hip_fail(e);
    const float bc1 = step_dev ? 0.f : (float)(1.0 - std::pow((double)beta1, step));
    const float bc2 = step_dev ? 0.f : (float)(1.0 - std::pow((double)beta2, step));
    hipLaunchKernelGGL(learn_finalize, dim3((uint32_t)(P->map.L * P->map.NI + 2)), dim3(kBlock), 0, hs, dc, nblk,
                       P->map, lp, nloss, N > 0 ? 1.0 / (double)N : 0.0, loss_dev, (float2 *)grad_coeffs,
                       (float *)coeffs_dev, adam_m, adam_v, lr, beta1, beta2, eps, bc1, bc2,
                       (const int32_t *)step_dev);
    e = hipGetLastError();
    return e == hipSuccess ? DPD_OK : hip_fail(e);
}

DPD_EXPORT dpd_status dpd_learn_step(dpd_plan *P, const dpd_plan *A, const dpd_plan *B, void *stream,
                                     void *coeffs_dev, float *adam_m, float *adam_v, int32_t step, float lr,
                                     float beta1, float beta2, float eps, const void *x, void *z, void *grad_y,
                                     int64_t rows, int64_t n, int64_t ld, float scale, float *loss_dev,
                                     void *grad_coeffs, void *ws, size_t ws_bytes)
{
    return learn_step(P, A, B, stream, coeffs_dev, adam_m, adam_v, step, nullptr, lr, beta1, beta2, eps, x, z,
                      grad_y, rows, n, ld, scale, loss_dev, grad_coeffs, ws, ws_bytes);
}

DPD_EXPORT dpd_status dpd_learn_step_dev(dpd_plan *P, const dpd_plan *A, const dpd_plan *B, void *stream,
                                         void *coeffs_dev, float *adam_m, float *adam_v, int32_t *step_dev, float lr,
                                         float beta1, float beta2, float eps, const void *x, void *z, void *grad_y,
                                         int64_t rows, int64_t n, int64_t ld, float scale, float *loss_dev,
                                         void *grad_coeffs, void *ws, size_t ws_bytes)
{
    if (step_dev == nullptr) return DPD_EINVAL;
    return learn_step(P, A, B, stream, coeffs_dev, adam_m, adam_v, 0, step_dev, lr, beta1, beta2, eps, x, z, grad_y,
                      rows, n, ld, scale, loss_dev, grad_coeffs, ws, ws_bytes);
}
